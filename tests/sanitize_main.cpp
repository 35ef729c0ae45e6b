// Test-only driver for the sanitizer build: the oracle (gp_oracle.c), the
// compiler's host lowering (lower.cpp) and the bounds-checked CPU replay of
// its tables (host_check.cpp) built with -fsanitize=address,undefined and run
// on the circuit files named on the command line. For every circuit it checks
// that the oracle gives the same per-fault signatures on one and on three
// threads, that the replayed lowering gives the oracle's signature for every
// fault, and that the files lowered as one merged batch replay the same way.
// Files whose name ends in ".bad" must be rejected by both the oracle and the
// lowering. Exit status 0 when all of that holds; sanitizer findings abort.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

extern "C" {
struct oracle_result {
  int64_t n_qubits, n_measurements, n_detectors, n_observables, n_channels;
  int64_t n_faults, n_empty, n_edges;
  int64_t* edge_off;
  int32_t* edge_bits;
  double* edge_q;
  int64_t n_edge_bits;
  int64_t* fault_off;
  int32_t* fault_bits;
  double* fault_p;
  int32_t* fault_channel;
  int32_t* fault_code;
};
int oracle_run_threads(const char* text, size_t len, const double* rates, int64_t n_rates, int keep_faults,
                       int64_t fault_stride, int n_threads, oracle_result** out);
void oracle_free(oracle_result* r);
const char* oracle_last_error(void);
int hc_run(const char* text, size_t len, const double* rates, size_t n_rates, uint64_t* off, uint32_t* bits,
           uint64_t bits_cap, uint32_t* src, uint32_t* code, uint64_t* stats, uint64_t max_faults);
int hc_run_batch(const char* const* texts, const size_t* lens, size_t n_texts, uint32_t slots, uint64_t* off,
                 uint32_t* bits, uint64_t bits_cap, uint32_t* src, uint32_t* code, uint64_t* stats,
                 uint64_t max_faults, uint32_t* fault_circuit);
const char* hc_error();
}

namespace {

using Sig = std::vector<uint32_t>;
using SigMap = std::map<std::pair<uint32_t, uint32_t>, Sig>;  // (channel, Pauli code) -> bits

int g_fail = 0;

void check(bool ok, const std::string& what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what.c_str());
    g_fail = 1;
  }
}

SigMap oracle_sigs(const std::string& text, int threads, int64_t* n_faults, int64_t* n_channels = nullptr) {
  oracle_result* r = nullptr;
  SigMap m;
  if (oracle_run_threads(text.data(), text.size(), nullptr, 0, 1, 1, threads, &r)) {
    check(false, std::string("oracle: ") + oracle_last_error());
    return m;
  }
  for (int64_t f = 0; f < r->n_faults; f++)
    m[{uint32_t(r->fault_channel[f]), uint32_t(r->fault_code[f])}] =
        Sig(r->fault_bits + r->fault_off[f], r->fault_bits + r->fault_off[f + 1]);
  *n_faults = r->n_faults;
  if (n_channels) *n_channels = r->n_channels;
  oracle_free(r);
  return m;
}

struct Replay {
  std::vector<uint64_t> off;
  std::vector<uint32_t> bits, src, code, circ;
  uint64_t stats[9] = {};
  explicit Replay(uint64_t cap) : off(cap + 1), bits(cap * 16), src(cap), code(cap), circ(cap) {}
  Sig sig(uint64_t p) const { return Sig(bits.begin() + off[p], bits.begin() + off[p + 1]); }
};

}  // namespace

int main(int argc, char** argv) {
  std::vector<std::string> good;
  for (int i = 1; i < argc; i++) {
    std::ifstream in(argv[i], std::ios::binary);
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string text = ss.str();
    const std::string name = argv[i];
    const bool bad = name.size() > 4 && name.compare(name.size() - 4, 4, ".bad") == 0;
    Replay rp(1 << 20);
    const int rc = hc_run(text.data(), text.size(), nullptr, 0, rp.off.data(), rp.bits.data(), rp.bits.size(),
                          rp.src.data(), rp.code.data(), rp.stats, 1 << 20);
    if (bad) {
      oracle_result* r = nullptr;
      const int orc = oracle_run_threads(text.data(), text.size(), nullptr, 0, 0, 1, 2, &r);
      if (r) oracle_free(r);
      check(rc != 0 && orc != 0, name + ": malformed circuit accepted");
      continue;
    }
    check(rc == 0, name + ": lowering/replay: " + (rc ? hc_error() : ""));
    if (rc) continue;
    int64_t nf1 = 0, nf3 = 0;
    const SigMap one = oracle_sigs(text, 1, &nf1);
    const SigMap three = oracle_sigs(text, 3, &nf3);
    check(nf1 == nf3 && one == three, name + ": oracle differs between one and three threads");
    check(uint64_t(nf1) == rp.stats[0], name + ": fault counts differ");
    for (uint64_t p = 0; p < rp.stats[0]; p++) {
      auto it = one.find({rp.src[p], rp.code[p]});
      if (it == one.end() || it->second != rp.sig(p)) {
        check(false, name + ": signature of fault at position " + std::to_string(p) + " differs");
        break;
      }
    }
    good.push_back(text);
    std::printf("%s: %lld faults ok\n", name.c_str(), (long long)nf1);
  }
  if (good.size() > 1) {
    std::vector<const char*> ptrs;
    std::vector<size_t> lens;
    for (const std::string& t : good) {
      ptrs.push_back(t.data());
      lens.push_back(t.size());
    }
    Replay rp(1 << 21);
    const int rc = hc_run_batch(ptrs.data(), lens.data(), good.size(), 16, rp.off.data(), rp.bits.data(),
                                rp.bits.size(), rp.src.data(), rp.code.data(), rp.stats, 1 << 21, rp.circ.data());
    check(rc == 0, std::string("batch replay: ") + (rc ? hc_error() : ""));
    if (rc == 0) {
      // positions run circuit by circuit; channels are numbered over the batch
      std::vector<SigMap> refs;
      std::vector<uint32_t> chan_base(good.size() + 1, 0);
      for (size_t k = 0; k < good.size(); k++) {
        int64_t nf = 0, nch = 0;
        refs.push_back(oracle_sigs(good[k], 2, &nf, &nch));
        chan_base[k + 1] = chan_base[k] + uint32_t(nch);
      }
      for (uint64_t p = 0; p < rp.stats[0]; p++) {
        const uint32_t k = rp.circ[p];
        auto it = refs[k].find({rp.src[p] - chan_base[k], rp.code[p]});
        if (it == refs[k].end() || it->second != rp.sig(p)) {
          check(false, "batch: signature of fault at position " + std::to_string(p) + " differs");
          break;
        }
      }
      std::printf("batch of %zu circuits: %llu faults ok\n", good.size(), (unsigned long long)rp.stats[0]);
    }
  }
  return g_fail;
}
