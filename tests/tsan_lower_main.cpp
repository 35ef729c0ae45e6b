// Test-only driver for the ThreadSanitizer build of the host lowering
// (lower.cpp built with -fsanitize=thread): lowers each circuit file named on
// the command line three times, twice into one kept set of tables and once
// into fresh ones, so that the tokenizer, channel-table and injection-list
// threads of large texts run against each other and against the scheduling
// thread. The kept and fresh tables must agree on their sizes and fault
// count. Files whose name ends in ".bad" must be rejected every time with
// the same message. Exit status 0 when all of that holds; a data race is
// reported by the sanitizer, which then fails the run.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "gp.h"
#include "lower.h"

int main(int argc, char** argv) {
  int failures = 0;
  for (int i = 1; i < argc; i++) {
    std::ifstream in(argv[i], std::ios::binary);
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string text = ss.str();
    const std::string name = argv[i];
    const bool bad = name.size() > 4 && name.compare(name.size() - 4, 4, ".bad") == 0;
    gp::Lowered kept, fresh;
    std::string first_msg;
    for (int rep = 0; rep < 3; rep++) {
      gp::Lowered& lw = rep < 2 ? kept : fresh;
      gp::LowerError err{0, ""};
      const int rc = gp::lower_circuit(text.data(), text.size(), nullptr, 0, 256, lw, err);
      if (bad) {
        if (rc == 0) {
          std::printf("FAIL %s: malformed circuit accepted\n", name.c_str());
          failures++;
        } else if (rep == 0) {
          first_msg = err.msg;
        } else if (err.msg != first_msg) {
          std::printf("FAIL %s: message changed: '%s' then '%s'\n", name.c_str(), first_msg.c_str(),
                      err.msg.c_str());
          failures++;
        }
      } else if (rc != 0) {
        std::printf("FAIL %s: %s\n", name.c_str(), err.msg.c_str());
        failures++;
      }
    }
    if (!bad && (kept.n_faults != fresh.n_faults || kept.ops.size() != fresh.ops.size() ||
                 kept.inj_word.size() != fresh.inj_word.size() || kept.chan_src.size() != fresh.chan_src.size())) {
      std::printf("FAIL %s: kept and fresh tables differ\n", name.c_str());
      failures++;
    }
    std::printf("%s %s%s\n", bad ? "rejected" : "lowered", name.c_str(), bad ? (": " + first_msg).c_str() : "");
  }
  return failures ? 1 : 0;
}
