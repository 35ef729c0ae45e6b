/*
 * gp_oracle.c -- plain CPU oracle for circuit-level decoding hypergraphs.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the product path. Only
 * the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load it; the compiler itself never calls into it, and it shares
 * no code, header, table or helper with the compiler.
 *
 * What it computes is the plain definition of the detector error model
 * (paper Sec. 2.1.4 "Detector error model", Sec. 2.1.5 "Error analysis",
 * Sec. 2.3.3 Eq. 3):
 *   1. every fault = (noise channel, one non-identity Pauli of that channel);
 *   2. its signature = the set of detectors and logical observables whose
 *      parity flips when that Pauli alone is inserted at the channel's place.
 *      The fault is tracked forward through the later operations (forward
 *      tracking, Sec. 2.1.5); the measurements it flips, combined with the
 *      DETECTOR / OBSERVABLE_INCLUDE definitions, give the signature;
 *   3. faults with equal signature form one equivalence class, whose
 *      probability is P = p_1 [+] p_2 [+] ... with a [+] b = a(1-b) + b(1-a)
 *      (Eq. 3), merged in fault order;
 *   4. the class with the empty signature is dropped.
 *
 * Per-fault probabilities (a reading; the paper does not state it): a
 * DEPOLARIZE1(r) channel is the composition of three independent channels X,
 * Y, Z each firing with probability p, and DEPOLARIZE2(r) of fifteen
 * independent two-qubit Pauli channels each firing with p. Matching the Pauli
 * transfer eigenvalues gives (1-2p)^2 = 1 - 4r/3 and (1-2p)^8 = 1 - 16r/15.
 * They are evaluated in rationalised forms that have no cancellation.
 * X_ERROR / Y_ERROR / Z_ERROR(r) give one fault with p = r.
 *
 * Arithmetic is IEEE binary64 throughout. The forward tracking of step 2 may
 * run on several threads, each over a contiguous range of fault ids; the
 * signatures are concatenated in fault order before step 3, which runs on one
 * thread, so the result does not depend on the thread count.
 */
#define _GNU_SOURCE
#include <ctype.h>
#include <pthread.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_PARSE (-2)
#define ORC_E_UNSUPPORTED (-3)
#define ORC_E_NOISE (-6)
#define ORC_E_OOM (-8)
#define ORC_E_ARG (-1)

static _Thread_local char g_err[512];

static int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

const char *oracle_last_error(void) { return g_err; }

/* ---------------------------------------------------------------- vectors */

typedef struct { int32_t *v; int64_t n, cap; } ivec;

static int ivec_push(ivec *a, int32_t x) {
  if (a->n == a->cap) {
    int64_t nc = a->cap ? a->cap * 2 : 64;
    int32_t *nv = (int32_t *)realloc(a->v, (size_t)nc * sizeof(int32_t));
    if (!nv) return ORC_E_OOM;
    a->v = nv;
    a->cap = nc;
  }
  a->v[a->n++] = x;
  return 0;
}

/* --------------------------------------------------------------- circuit */

enum {
  K_H = 1, K_S, K_SQRTX, K_CX, K_CZ, K_SWAP,
  K_R, K_RX, K_M, K_MX, K_MR, K_MRX
};

enum { N_X = 1, N_Y, N_Z, N_DEP1, N_DEP2 };

typedef struct { int kind, q0, q1, m; } op_t;

typedef struct {
  int kind, qa, qb;
  int64_t at;  /* the fault acts just before elementary operation `at` */
  double rate;
} chan_t;

typedef struct {
  op_t *ops; int64_t nops, capops;
  chan_t *ch; int64_t nch, capch;
  int nq;
  int64_t nmeas;
  int ndet, nobs;
  /* (measurement, code) pairs; code >= 0 detector, code < 0 observable -(k+1) */
  int64_t *pm; int32_t *pc; int64_t np, capp;
  /* per-qubit operation lists */
  int64_t *qoff; int64_t *qops;
  /* leaves: measurement -> sorted list of signature bits */
  int64_t *loff; int32_t *lbits;
} circ_t;

static void circ_free(circ_t *c) {
  free(c->ops); free(c->ch); free(c->pm); free(c->pc);
  free(c->qoff); free(c->qops); free(c->loff); free(c->lbits);
  memset(c, 0, sizeof *c);
}

static int add_op(circ_t *c, int kind, int q0, int q1, int m) {
  if (c->nops == c->capops) {
    int64_t nc = c->capops ? c->capops * 2 : 256;
    op_t *n = (op_t *)realloc(c->ops, (size_t)nc * sizeof(op_t));
    if (!n) return ORC_E_OOM;
    c->ops = n; c->capops = nc;
  }
  c->ops[c->nops++] = (op_t){kind, q0, q1, m};
  if (q0 >= c->nq) c->nq = q0 + 1;
  if (q1 >= c->nq) c->nq = q1 + 1;
  return 0;
}

static int add_chan(circ_t *c, int kind, int qa, int qb, double rate) {
  if (c->nch == c->capch) {
    int64_t nc = c->capch ? c->capch * 2 : 256;
    chan_t *n = (chan_t *)realloc(c->ch, (size_t)nc * sizeof(chan_t));
    if (!n) return ORC_E_OOM;
    c->ch = n; c->capch = nc;
  }
  c->ch[c->nch++] = (chan_t){kind, qa, qb, c->nops, rate};
  if (qa >= c->nq) c->nq = qa + 1;
  if (qb >= c->nq) c->nq = qb + 1;
  return 0;
}

static int add_pair(circ_t *c, int64_t m, int32_t code) {
  if (c->np == c->capp) {
    int64_t nc = c->capp ? c->capp * 2 : 256;
    int64_t *a = (int64_t *)realloc(c->pm, (size_t)nc * sizeof(int64_t));
    if (!a) return ORC_E_OOM;
    c->pm = a;
    int32_t *b = (int32_t *)realloc(c->pc, (size_t)nc * sizeof(int32_t));
    if (!b) return ORC_E_OOM;
    c->pc = b;
    c->capp = nc;
  }
  c->pm[c->np] = m;
  c->pc[c->np] = code;
  c->np++;
  return 0;
}

/* ---------------------------------------------------------------- parser */

typedef struct { const char *name; int cls, kind; } gate_def;
enum { C_1Q = 1, C_2Q, C_MEAS, C_RESET, C_NOISE1, C_NOISE2, C_DET, C_OBS, C_SKIP, C_PAULI };

static const gate_def GATES[] = {
  {"H", C_1Q, K_H}, {"H_XZ", C_1Q, K_H},
  {"S", C_1Q, K_S}, {"S_DAG", C_1Q, K_S}, {"SQRT_Z", C_1Q, K_S}, {"SQRT_Z_DAG", C_1Q, K_S},
  {"SQRT_X", C_1Q, K_SQRTX}, {"SQRT_X_DAG", C_1Q, K_SQRTX},
  {"I", C_PAULI, 0}, {"X", C_PAULI, 0}, {"Y", C_PAULI, 0}, {"Z", C_PAULI, 0},
  {"CX", C_2Q, K_CX}, {"CNOT", C_2Q, K_CX}, {"ZCX", C_2Q, K_CX},
  {"CZ", C_2Q, K_CZ}, {"ZCZ", C_2Q, K_CZ}, {"SWAP", C_2Q, K_SWAP},
  {"R", C_RESET, K_R}, {"RZ", C_RESET, K_R}, {"RX", C_RESET, K_RX},
  {"M", C_MEAS, K_M}, {"MZ", C_MEAS, K_M}, {"MX", C_MEAS, K_MX},
  {"MR", C_MEAS, K_MR}, {"MRZ", C_MEAS, K_MR}, {"MRX", C_MEAS, K_MRX},
  {"X_ERROR", C_NOISE1, N_X}, {"Y_ERROR", C_NOISE1, N_Y}, {"Z_ERROR", C_NOISE1, N_Z},
  {"DEPOLARIZE1", C_NOISE1, N_DEP1}, {"DEPOLARIZE2", C_NOISE2, N_DEP2},
  {"DETECTOR", C_DET, 0}, {"OBSERVABLE_INCLUDE", C_OBS, 0},
  {"TICK", C_SKIP, 0}, {"QUBIT_COORDS", C_SKIP, 0}, {"SHIFT_COORDS", C_SKIP, 0},
  {NULL, 0, 0}};

#define MAXTOK 1024

static int parse(const char *text, size_t len, circ_t *c) {
  size_t pos = 0;
  int lineno = 0;
  char name[64];
  double args[16];
  int64_t *tg = NULL;   /* targets: a qubit, or k for rec[-k] when isrec is set */
  int *isrec = NULL;
  int64_t ntg = 0, captg = 0;
  int rc = 0;
  while (pos < len) {
    size_t e = pos;
    while (e < len && text[e] != '\n') e++;
    lineno++;
    /* copy the line without its comment */
    size_t ll = e - pos;
    const char *ln = text + pos;
    size_t cut = 0;
    while (cut < ll && ln[cut] != '#') cut++;
    pos = e + 1;
    size_t i = 0;
    while (i < cut && isspace((unsigned char)ln[i])) i++;
    if (i == cut) continue;
    /* instruction name */
    int nl = 0;
    while (i < cut && !isspace((unsigned char)ln[i]) && ln[i] != '(') {
      if (nl < 63) name[nl++] = (char)toupper((unsigned char)ln[i]);
      i++;
    }
    name[nl] = 0;
    if (!strcmp(name, "REPEAT") || !strcmp(name, "{") || !strcmp(name, "}")) {
      rc = fail(ORC_E_UNSUPPORTED, "line %d: REPEAT blocks are not supported", lineno);
      goto done;
    }
    int nargs = 0;
    if (i < cut && ln[i] == '(') {
      i++;
      for (;;) {
        while (i < cut && isspace((unsigned char)ln[i])) i++;
        if (i < cut && ln[i] == ')') { i++; break; }
        char buf[64];
        int bl = 0;
        while (i < cut && ln[i] != ',' && ln[i] != ')' && bl < 63) buf[bl++] = ln[i++];
        buf[bl] = 0;
        char *endp;
        double v = strtod(buf, &endp);
        if (endp == buf || nargs >= 16) { rc = fail(ORC_E_PARSE, "line %d: bad argument", lineno); goto done; }
        args[nargs++] = v;
        if (i < cut && ln[i] == ',') i++;
        else if (i >= cut) { rc = fail(ORC_E_PARSE, "line %d: unterminated arguments", lineno); goto done; }
      }
    }
    /* targets */
    ntg = 0;
    for (;;) {
      while (i < cut && isspace((unsigned char)ln[i])) i++;
      if (i >= cut) break;
      size_t s = i;
      while (i < cut && !isspace((unsigned char)ln[i])) i++;
      char tok[MAXTOK];
      size_t tl = i - s;
      if (tl >= MAXTOK) { rc = fail(ORC_E_PARSE, "line %d: target too long", lineno); goto done; }
      memcpy(tok, ln + s, tl);
      tok[tl] = 0;
      if (ntg == captg) {
        captg = captg ? captg * 2 : 64;
        tg = (int64_t *)realloc(tg, (size_t)captg * sizeof(int64_t));
        isrec = (int *)realloc(isrec, (size_t)captg * sizeof(int));
        if (!tg || !isrec) { rc = fail(ORC_E_OOM, "out of memory"); goto done; }
      }
      if (!strncmp(tok, "rec[-", 5) && tok[tl - 1] == ']') {
        char *endp;
        long long k = strtoll(tok + 5, &endp, 10);
        if (*endp != ']' || k <= 0) { rc = fail(ORC_E_PARSE, "line %d: bad record target %s", lineno, tok); goto done; }
        tg[ntg] = k;
        isrec[ntg] = 1;
      } else {
        char *endp;
        long long q = strtoll(tok, &endp, 10);
        if (*endp != 0 || endp == tok || q < 0 || q > (1LL << 28)) {
          rc = fail(ORC_E_UNSUPPORTED, "line %d: unsupported target %s", lineno, tok);
          goto done;
        }
        tg[ntg] = q;
        isrec[ntg] = 0;
      }
      ntg++;
    }
    const gate_def *g = NULL;
    for (int k = 0; GATES[k].name; k++)
      if (!strcmp(GATES[k].name, name)) { g = &GATES[k]; break; }
    if (!g) { rc = fail(ORC_E_UNSUPPORTED, "line %d: unsupported instruction %s", lineno, name); goto done; }
    int needs_qubits = (g->cls == C_1Q || g->cls == C_2Q || g->cls == C_MEAS || g->cls == C_RESET ||
                        g->cls == C_NOISE1 || g->cls == C_NOISE2 || g->cls == C_PAULI);
    if (needs_qubits) {
      for (int64_t k = 0; k < ntg; k++)
        if (isrec[k]) { rc = fail(ORC_E_PARSE, "line %d: record target on %s", lineno, name); goto done; }
    }
    if ((g->cls == C_1Q || g->cls == C_2Q || g->cls == C_MEAS || g->cls == C_RESET || g->cls == C_PAULI) && nargs) {
      rc = fail(ORC_E_UNSUPPORTED, "line %d: arguments on %s are not supported", lineno, name);
      goto done;
    }
    switch (g->cls) {
      case C_PAULI:
        /* Pauli gates commute with every Pauli fault up to sign: no effect. */
        for (int64_t k = 0; k < ntg; k++)
          if (tg[k] >= c->nq) c->nq = (int)tg[k] + 1;
        break;
      case C_1Q:
      case C_RESET:
        for (int64_t k = 0; k < ntg; k++)
          if ((rc = add_op(c, g->kind, (int)tg[k], -1, -1))) goto done;
        break;
      case C_2Q:
        if (ntg % 2) { rc = fail(ORC_E_PARSE, "line %d: odd target count for %s", lineno, name); goto done; }
        for (int64_t k = 0; k < ntg; k += 2) {
          if (tg[k] == tg[k + 1]) { rc = fail(ORC_E_PARSE, "line %d: repeated qubit in %s", lineno, name); goto done; }
          if ((rc = add_op(c, g->kind, (int)tg[k], (int)tg[k + 1], -1))) goto done;
        }
        break;
      case C_MEAS:
        for (int64_t k = 0; k < ntg; k++)
          if ((rc = add_op(c, g->kind, (int)tg[k], -1, (int)(c->nmeas++)))) goto done;
        break;
      case C_NOISE1:
      case C_NOISE2: {
        if (nargs != 1) { rc = fail(ORC_E_PARSE, "line %d: %s takes one probability", lineno, name); goto done; }
        double r = args[0];
        double lim = g->kind == N_DEP1 ? 0.75 : g->kind == N_DEP2 ? 15.0 / 16.0 : 0.5;
        if (!(r >= 0.0 && r <= lim)) { rc = fail(ORC_E_NOISE, "line %d: rate %g out of range", lineno, r); goto done; }
        if (g->cls == C_NOISE1) {
          for (int64_t k = 0; k < ntg; k++)
            if ((rc = add_chan(c, g->kind, (int)tg[k], -1, r))) goto done;
        } else {
          if (ntg % 2) { rc = fail(ORC_E_PARSE, "line %d: odd target count for %s", lineno, name); goto done; }
          for (int64_t k = 0; k < ntg; k += 2) {
            if (tg[k] == tg[k + 1]) { rc = fail(ORC_E_PARSE, "line %d: repeated qubit in %s", lineno, name); goto done; }
            if ((rc = add_chan(c, g->kind, (int)tg[k], (int)tg[k + 1], r))) goto done;
          }
        }
        break;
      }
      case C_DET:
      case C_OBS: {
        int32_t code;
        if (g->cls == C_DET) {
          code = c->ndet++;
        } else {
          if (nargs != 1 || args[0] < 0 || args[0] != floor(args[0]) || args[0] > 1e6) {
            rc = fail(ORC_E_PARSE, "line %d: OBSERVABLE_INCLUDE needs an index", lineno);
            goto done;
          }
          int k = (int)args[0];
          if (k + 1 > c->nobs) c->nobs = k + 1;
          code = -(k + 1);
        }
        for (int64_t k = 0; k < ntg; k++) {
          if (!isrec[k]) { rc = fail(ORC_E_PARSE, "line %d: %s takes record targets", lineno, name); goto done; }
          int64_t m = c->nmeas - tg[k];
          if (m < 0) { rc = fail(ORC_E_PARSE, "line %d: record looks back too far", lineno); goto done; }
          if ((rc = add_pair(c, m, code))) goto done;
        }
        break;
      }
      default:
        break;
    }
  }
done:
  free(tg);
  free(isrec);
  return rc;
}

/* Sort (m, code) pairs and cancel duplicates pairwise: a measurement that a
 * detector or observable lists an even number of times does not belong to it. */
static int cmp_pair_idx(const void *a, const void *b, void *ctx) {
  const circ_t *c = (const circ_t *)ctx;
  int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
  if (c->pm[i] != c->pm[j]) return c->pm[i] < c->pm[j] ? -1 : 1;
  if (c->pc[i] != c->pc[j]) return c->pc[i] < c->pc[j] ? -1 : 1;
  return 0;
}

static int build_tables(circ_t *c) {
  int64_t M = c->nmeas;
  int64_t *idx = (int64_t *)malloc((size_t)(c->np ? c->np : 1) * sizeof(int64_t));
  c->loff = (int64_t *)calloc((size_t)M + 1, sizeof(int64_t));
  c->lbits = (int32_t *)malloc((size_t)(c->np ? c->np : 1) * sizeof(int32_t));
  if (!idx || !c->loff || !c->lbits) { free(idx); return fail(ORC_E_OOM, "out of memory"); }
  for (int64_t i = 0; i < c->np; i++) idx[i] = i;
  qsort_r(idx, (size_t)c->np, sizeof(int64_t), cmp_pair_idx, c);
  /* count surviving pairs per measurement */
  int64_t nb = 0;
  int64_t i = 0;
  while (i < c->np) {
    int64_t j = i;
    while (j < c->np && c->pm[idx[j]] == c->pm[idx[i]] && c->pc[idx[j]] == c->pc[idx[i]]) j++;
    if ((j - i) % 2 == 1) {
      int32_t code = c->pc[idx[i]];
      int32_t bit = code >= 0 ? code : c->ndet + (-code - 1);
      c->loff[c->pm[idx[i]] + 1]++;
      c->lbits[nb++] = bit;
    }
    i = j;
  }
  for (int64_t m = 0; m < M; m++) c->loff[m + 1] += c->loff[m];
  /* bits were appended in (m, code) order, so each measurement's slice is
   * contiguous; sort each slice (observable codes were negative) */
  for (int64_t m = 0; m < M; m++) {
    for (int64_t a = c->loff[m] + 1; a < c->loff[m + 1]; a++) {
      int32_t v = c->lbits[a];
      int64_t b = a - 1;
      while (b >= c->loff[m] && c->lbits[b] > v) { c->lbits[b + 1] = c->lbits[b]; b--; }
      c->lbits[b + 1] = v;
    }
  }
  free(idx);
  /* per-qubit operation lists */
  c->qoff = (int64_t *)calloc((size_t)c->nq + 1, sizeof(int64_t));
  c->qops = (int64_t *)malloc((size_t)(2 * c->nops + 1) * sizeof(int64_t));
  if (!c->qoff || !c->qops) return fail(ORC_E_OOM, "out of memory");
  for (int64_t k = 0; k < c->nops; k++) {
    c->qoff[c->ops[k].q0 + 1]++;
    if (c->ops[k].q1 >= 0) c->qoff[c->ops[k].q1 + 1]++;
  }
  for (int q = 0; q < c->nq; q++) c->qoff[q + 1] += c->qoff[q];
  int64_t *fill = (int64_t *)malloc((size_t)(c->nq + 1) * sizeof(int64_t));
  if (!fill) return fail(ORC_E_OOM, "out of memory");
  memcpy(fill, c->qoff, (size_t)(c->nq + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < c->nops; k++) {
    c->qops[fill[c->ops[k].q0]++] = k;
    if (c->ops[k].q1 >= 0) c->qops[fill[c->ops[k].q1]++] = k;
  }
  free(fill);
  return 0;
}

/* -------------------------------------------------------- fault probability */

/* One fault of a DEPOLARIZE1(r) channel: p with (1-2p)^2 = 1 - 4r/3, i.e.
 * p = (1 - sqrt(1-x))/2 = x / (2 (1 + sqrt(1-x))), x = 4r/3. */
static double split_dep1(double r) {
  double x = 4.0 * r / 3.0;
  return x / (2.0 * (1.0 + sqrt(1.0 - x)));
}

/* One fault of a DEPOLARIZE2(r) channel: p with (1-2p)^8 = 1 - 16r/15. With
 * s = (1-x)^(1/8), 1 - s = x / ((1+s)(1+s^2)(1+s^4)), x = 16r/15. */
static double split_dep2(double r) {
  double x = 16.0 * r / 15.0;
  double s4 = sqrt(1.0 - x);
  double s2 = sqrt(s4);
  double s1 = sqrt(s2);
  return x / (2.0 * (1.0 + s1) * (1.0 + s2) * (1.0 + s4));
}

/* Pauli codes: bit0 = x on qa, bit1 = z on qa, bit2 = x on qb, bit3 = z on qb. */
static int chan_faults(int kind, int codes[15]) {
  switch (kind) {
    case N_X: codes[0] = 1; return 1;
    case N_Y: codes[0] = 3; return 1;
    case N_Z: codes[0] = 2; return 1;
    case N_DEP1: codes[0] = 1; codes[1] = 3; codes[2] = 2; return 3;
    case N_DEP2: {
      /* single-qubit Paulis in the order I, X, Y, Z -> (x, z) bit pairs */
      static const int pz[4] = {0, 1, 3, 2};
      int n = 0;
      for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
          if (a || b) codes[n++] = pz[a] | (pz[b] << 2);
      return n;
    }
  }
  return 0;
}

/* Correlation levels, Table 1: the two-qubit Paulis each level adds, by name
 * (first letter = first target). One-qubit channels follow the same split:
 * X and Z at level 0, Y from level 1. */
static const char *const LEVEL_NAMES[3][6] = {
    {"IX", "IZ", "XI", "XX", "ZI", "ZZ"},
    {"IY", "XZ", "YI", "ZX", NULL, NULL},
    {"XY", "YX", "YY", "YZ", "ZY", NULL},
};

static char pauli_letter(int xz) { return "IXZY"[xz & 3]; }

static int pauli_level_of(int kind, int code) {
  char name[3] = {0, 0, 0};
  if (kind == N_DEP2) {
    name[0] = pauli_letter(code & 3);
    name[1] = pauli_letter((code >> 2) & 3);
  } else {
    /* a one-qubit Pauli P is ranked like IP */
    name[0] = 'I';
    name[1] = pauli_letter(code & 3);
  }
  for (int l = 0; l < 3; l++)
    for (int k = 0; k < 6 && LEVEL_NAMES[l][k]; k++)
      if (!strcmp(name, LEVEL_NAMES[l][k])) return l;
  return 3;
}

static int g_level = 2;

static double fault_p(int kind, double r) {
  switch (kind) {
    case N_DEP1: return split_dep1(r);
    case N_DEP2: return split_dep2(r);
    default: return r;
  }
}

/* ----------------------------------------------------- forward tracking */

typedef struct { int q, x, z; int64_t ptr; } entry_t;

typedef struct {
  entry_t *e; int ne, cap;
  int64_t *flip; int64_t nflip, capflip;
  unsigned char *mark; int32_t *touched; int64_t ntouched;
  ivec sig;
} scratch_t;

static int64_t lower_bound(const int64_t *a, int64_t lo, int64_t hi, int64_t key) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

static int find_entry(scratch_t *s, int q) {
  for (int i = 0; i < s->ne; i++)
    if (s->e[i].q == q) return i;
  return -1;
}

static int push_entry(scratch_t *s, const circ_t *c, int q, int x, int z, int64_t at) {
  if (s->ne == s->cap) {
    int nc = s->cap ? s->cap * 2 : 16;
    entry_t *n = (entry_t *)realloc(s->e, (size_t)nc * sizeof(entry_t));
    if (!n) return -1;
    s->e = n; s->cap = nc;
  }
  entry_t *en = &s->e[s->ne];
  en->q = q; en->x = x; en->z = z;
  en->ptr = lower_bound(c->qops, c->qoff[q], c->qoff[q + 1], at);
  return s->ne++;
}

static int toggle_flip(scratch_t *s, int64_t m) {
  for (int64_t i = 0; i < s->nflip; i++)
    if (s->flip[i] == m) { s->flip[i] = s->flip[--s->nflip]; return 0; }
  if (s->nflip == s->capflip) {
    int64_t nc = s->capflip ? s->capflip * 2 : 16;
    int64_t *n = (int64_t *)realloc(s->flip, (size_t)nc * sizeof(int64_t));
    if (!n) return -1;
    s->flip = n; s->capflip = nc;
  }
  s->flip[s->nflip++] = m;
  return 0;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Track one fault forward; leave its sorted signature in s->sig. */
static int track_fault(const circ_t *c, const chan_t *ch, int code, scratch_t *s) {
  s->ne = 0;
  s->nflip = 0;
  if ((code & 3) && push_entry(s, c, ch->qa, code & 1, (code >> 1) & 1, ch->at) < 0) return ORC_E_OOM;
  if ((code >> 2) && push_entry(s, c, ch->qb, (code >> 2) & 1, (code >> 3) & 1, ch->at) < 0) return ORC_E_OOM;
  for (;;) {
    /* the next operation, in program order, that touches a frame qubit */
    int best = -1;
    int64_t bestop = INT64_MAX;
    for (int i = 0; i < s->ne; i++) {
      const entry_t *en = &s->e[i];
      if (en->ptr < c->qoff[en->q + 1]) {
        int64_t k = c->qops[en->ptr];
        if (k < bestop) { bestop = k; best = i; }
      }
    }
    if (best < 0) break;
    const op_t *op = &c->ops[bestop];
    entry_t *a = &s->e[best];
    switch (op->kind) {
      case K_H: { int t = a->x; a->x = a->z; a->z = t; a->ptr++; break; }
      case K_S: a->z ^= a->x; a->ptr++; break;          /* X -> Y, Z -> Z */
      case K_SQRTX: a->x ^= a->z; a->ptr++; break;      /* Z -> Y, X -> X */
      case K_R: case K_RX: a->x = 0; a->z = 0; a->ptr++; break;
      case K_M: if (a->x && toggle_flip(s, op->m)) return ORC_E_OOM; a->ptr++; break;
      case K_MX: if (a->z && toggle_flip(s, op->m)) return ORC_E_OOM; a->ptr++; break;
      case K_MR:
        if (a->x && toggle_flip(s, op->m)) return ORC_E_OOM;
        a->x = 0; a->z = 0; a->ptr++; break;
      case K_MRX:
        if (a->z && toggle_flip(s, op->m)) return ORC_E_OOM;
        a->x = 0; a->z = 0; a->ptr++; break;
      case K_CX: case K_CZ: case K_SWAP: {
        int qa = a->q;
        int other = op->q0 == qa ? op->q1 : op->q0;
        int j = find_entry(s, other);
        if (j < 0) {
          j = push_entry(s, c, other, 0, 0, bestop);
          if (j < 0) return ORC_E_OOM;
        }
        entry_t *p0 = &s->e[find_entry(s, op->q0)];
        entry_t *p1 = &s->e[find_entry(s, op->q1)];
        if (op->kind == K_CX) {          /* control q0, target q1 */
          p1->x ^= p0->x;
          p0->z ^= p1->z;
        } else if (op->kind == K_CZ) {
          int x0 = p0->x, x1 = p1->x;
          p0->z ^= x1;
          p1->z ^= x0;
        } else {
          int tx = p0->x, tz = p0->z;
          p0->x = p1->x; p0->z = p1->z;
          p1->x = tx; p1->z = tz;
        }
        p0->ptr++;
        p1->ptr++;
        break;
      }
      default:
        return fail(ORC_E_ARG, "internal: bad operation");
    }
    /* drop qubits whose frame component vanished */
    for (int i = 0; i < s->ne;) {
      if (!s->e[i].x && !s->e[i].z) s->e[i] = s->e[--s->ne];
      else i++;
    }
  }
  /* signature = XOR of the leaves of the flipped measurements */
  s->ntouched = 0;
  for (int64_t i = 0; i < s->nflip; i++) {
    int64_t m = s->flip[i];
    for (int64_t k = c->loff[m]; k < c->loff[m + 1]; k++) {
      int32_t b = c->lbits[k];
      if (!s->mark[b]) s->touched[s->ntouched++] = b;
      s->mark[b] ^= 1;
    }
  }
  /* a bit that went 0 -> 1 -> 0 -> 1 sits in `touched` twice: collect the
   * set bits, clear every mark, then sort and drop repeats */
  s->sig.n = 0;
  for (int64_t i = 0; i < s->ntouched; i++) {
    int32_t b = s->touched[i];
    if (s->mark[b] && ivec_push(&s->sig, b)) return ORC_E_OOM;
  }
  for (int64_t i = 0; i < s->ntouched; i++) s->mark[s->touched[i]] = 0;
  if (s->sig.n > 1) qsort(s->sig.v, (size_t)s->sig.n, sizeof(int32_t), cmp_i32);
  int64_t w = 0;
  for (int64_t i = 0; i < s->sig.n; i++)
    if (w == 0 || s->sig.v[w - 1] != s->sig.v[i]) s->sig.v[w++] = s->sig.v[i];
  s->sig.n = w;
  return 0;
}

/* ------------------------------------------------------------ result */

typedef struct oracle_result {
  int64_t n_qubits, n_measurements, n_detectors, n_observables, n_channels;
  int64_t n_faults;       /* faults analysed */
  int64_t n_empty;        /* faults with an empty signature */
  int64_t n_edges;
  int64_t *edge_off;      /* n_edges + 1 */
  int32_t *edge_bits;     /* detector indices, then D + observable index */
  double *edge_q;
  int64_t n_edge_bits;
  /* per fault (only when requested) */
  int64_t *fault_off;
  int32_t *fault_bits;
  double *fault_p;
  int32_t *fault_channel;
  int32_t *fault_code;
} oracle_result;

void oracle_free(oracle_result *r) {
  if (!r) return;
  free(r->edge_off); free(r->edge_bits); free(r->edge_q);
  free(r->fault_off); free(r->fault_bits); free(r->fault_p);
  free(r->fault_channel); free(r->fault_code);
  free(r);
}

typedef struct {
  const int64_t *off;
  const int32_t *bits;
} sigctx_t;

static int cmp_fault(const void *pa, const void *pb, void *ctx) {
  const sigctx_t *g = (const sigctx_t *)ctx;
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  int64_t la = g->off[a + 1] - g->off[a], lb = g->off[b + 1] - g->off[b];
  const int32_t *x = g->bits + g->off[a], *y = g->bits + g->off[b];
  int64_t n = la < lb ? la : lb;
  for (int64_t i = 0; i < n; i++)
    if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
  if (la != lb) return la < lb ? -1 : 1;
  return (a > b) - (a < b);
}

/* One thread's share of the forward tracking: faults [lo, hi) of the
 * selected list, in order; their signatures are appended to `pool` with
 * offsets in `off` (relative to this share). */
typedef struct {
  const circ_t *c;
  const int64_t *fch;   /* selected faults: channel */
  const int32_t *fcode; /* and Pauli code */
  int64_t lo, hi;
  int64_t nbits;
  int64_t *off;         /* hi - lo + 1 */
  ivec pool;
  int rc;
  char err[512];
} share_t;

static void *track_share(void *arg) {
  share_t *sh = (share_t *)arg;
  scratch_t s;
  memset(&s, 0, sizeof s);
  s.mark = (unsigned char *)calloc((size_t)sh->nbits + 1, 1);
  s.touched = (int32_t *)malloc(((size_t)sh->nbits + 1) * sizeof(int32_t));
  sh->off = (int64_t *)malloc((size_t)(sh->hi - sh->lo + 1) * sizeof(int64_t));
  if (!s.mark || !s.touched || !sh->off) {
    sh->rc = ORC_E_OOM;
  } else {
    for (int64_t i = sh->lo; i < sh->hi && !sh->rc; i++) {
      sh->off[i - sh->lo] = sh->pool.n;
      int rc = track_fault(sh->c, &sh->c->ch[sh->fch[i]], sh->fcode[i], &s);
      if (rc) {
        sh->rc = rc;
        snprintf(sh->err, sizeof sh->err, "%s", g_err);  /* this thread's message */
        break;
      }
      for (int64_t b = 0; b < s.sig.n; b++)
        if (ivec_push(&sh->pool, s.sig.v[b])) { sh->rc = ORC_E_OOM; break; }
    }
    if (!sh->rc) sh->off[sh->hi - sh->lo] = sh->pool.n;
  }
  free(s.e); free(s.flip); free(s.mark); free(s.touched); free(s.sig.v);
  return NULL;
}

/*
 * oracle_run: compile `text` (Stim-format subset) to its hypergraph.
 *   rates / n_rates : optional per-channel rates (channel order = program
 *                     order x target group); NULL keeps the rates in the text.
 *   keep_faults     : also return each analysed fault's signature.
 *   fault_stride    : analyse only faults whose id is a multiple of this
 *                     (1 = all); used to time the oracle on a bounded sample.
 * oracle_run_threads: the same with the forward tracking on `n_threads`
 * threads (contiguous fault ranges); identical output for any thread count.
 */
int oracle_run_threads(const char *text, size_t len, const double *rates, int64_t n_rates,
                       int keep_faults, int64_t fault_stride, int n_threads, oracle_result **out);

int oracle_run(const char *text, size_t len, const double *rates, int64_t n_rates,
               int keep_faults, int64_t fault_stride, oracle_result **out) {
  return oracle_run_threads(text, len, rates, n_rates, keep_faults, fault_stride, 1, out);
}

int oracle_run_threads(const char *text, size_t len, const double *rates, int64_t n_rates,
                       int keep_faults, int64_t fault_stride, int n_threads, oracle_result **out) {
  *out = NULL;
  if (fault_stride < 1) return fail(ORC_E_ARG, "fault_stride must be >= 1");
  if (n_threads < 1 || n_threads > 1024) return fail(ORC_E_ARG, "n_threads must be in [1, 1024]");
  circ_t c;
  memset(&c, 0, sizeof c);
  int rc = parse(text, len, &c);
  if (rc) { circ_free(&c); return rc; }
  if (rates) {
    if (n_rates != c.nch) {
      circ_free(&c);
      return fail(ORC_E_NOISE, "rate array has %lld entries, circuit has %lld channels",
                  (long long)n_rates, (long long)c.nch);
    }
    for (int64_t k = 0; k < c.nch; k++) {
      double r = rates[k];
      int kind = c.ch[k].kind;
      double lim = kind == N_DEP1 ? 0.75 : kind == N_DEP2 ? 15.0 / 16.0 : 0.5;
      if (!(r >= 0.0 && r <= lim)) { circ_free(&c); return fail(ORC_E_NOISE, "rate %g out of range", r); }
      c.ch[k].rate = r;
    }
  }
  if ((rc = build_tables(&c))) { circ_free(&c); return rc; }
  int64_t nbits = (int64_t)c.ndet + c.nobs;

  oracle_result *res = (oracle_result *)calloc(1, sizeof *res);
  ivec pool = {0};
  int64_t *foff = NULL;
  double *fp = NULL;
  int32_t *fch = NULL, *fcode = NULL;
  int64_t *fch64 = NULL;
  share_t *sh = NULL;
  int64_t nf = 0, capf = 0;
  if (!res) { rc = fail(ORC_E_OOM, "out of memory"); goto fin; }

  /* the faults analysed, in fault order: (channel, Pauli code, probability) */
  {
    int64_t fid = 0;
    int codes[15];
    for (int64_t k = 0; k < c.nch; k++) {
      int nfc = chan_faults(c.ch[k].kind, codes);
      double p = fault_p(c.ch[k].kind, c.ch[k].rate);
      for (int j = 0; j < nfc; j++) {
        /* faults above the correlation level are not part of the model */
        if (pauli_level_of(c.ch[k].kind, codes[j]) > g_level) continue;
        if ((fid++) % fault_stride) continue;
        if (nf == capf) {
          capf = capf ? capf * 2 : 1024;
          fp = (double *)realloc(fp, (size_t)capf * sizeof(double));
          fch = (int32_t *)realloc(fch, (size_t)capf * sizeof(int32_t));
          fch64 = (int64_t *)realloc(fch64, (size_t)capf * sizeof(int64_t));
          fcode = (int32_t *)realloc(fcode, (size_t)capf * sizeof(int32_t));
          if (!fp || !fch || !fch64 || !fcode) { rc = fail(ORC_E_OOM, "out of memory"); goto fin; }
        }
        fp[nf] = p;
        fch[nf] = (int32_t)k;
        fch64[nf] = k;
        fcode[nf] = codes[j];
        nf++;
      }
    }
  }

  /* stage: one forward-tracking pass per fault, over contiguous fault
   * ranges, then the signatures concatenated in fault order */
  {
    int T = n_threads;
    if (T > 1 && nf < 4096 * (int64_t)T) T = (int)(nf / 4096 > 1 ? nf / 4096 : 1);
    sh = (share_t *)calloc((size_t)T, sizeof *sh);
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof *th);
    int *started = (int *)calloc((size_t)T, sizeof *started);
    if (!sh || !th || !started) { free(th); free(started); rc = fail(ORC_E_OOM, "out of memory"); goto fin; }
    for (int t = 0; t < T; t++) {
      sh[t].c = &c;
      sh[t].fch = fch64;
      sh[t].fcode = fcode;
      sh[t].lo = nf * t / T;
      sh[t].hi = nf * (t + 1) / T;
      sh[t].nbits = nbits;
    }
    for (int t = 1; t < T; t++) started[t] = pthread_create(&th[t], NULL, track_share, &sh[t]) == 0;
    track_share(&sh[0]);
    for (int t = 1; t < T; t++) {
      if (started[t]) pthread_join(th[t], NULL);
      else track_share(&sh[t]);  /* could not start a thread: run its share here */
    }
    free(th);
    free(started);
    int64_t total = 0;
    for (int t = 0; t < T; t++) {
      if (sh[t].rc && !rc)
        rc = sh[t].rc == ORC_E_OOM ? fail(ORC_E_OOM, "out of memory") : fail(sh[t].rc, "%s", sh[t].err);
      total += sh[t].pool.n;
    }
    if (!rc) {
      foff = (int64_t *)malloc((size_t)(nf + 1) * sizeof(int64_t));
      pool.v = (int32_t *)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
      pool.cap = total ? total : 1;
      if (!foff || !pool.v) rc = fail(ORC_E_OOM, "out of memory");
    }
    if (!rc) {
      for (int t = 0; t < T; t++) {
        for (int64_t i = sh[t].lo; i < sh[t].hi; i++) foff[i] = pool.n + sh[t].off[i - sh[t].lo];
        if (sh[t].pool.n) memcpy(pool.v + pool.n, sh[t].pool.v, (size_t)sh[t].pool.n * sizeof(int32_t));
        pool.n += sh[t].pool.n;
      }
      foff[nf] = pool.n;
    }
    for (int t = 0; t < T; t++) { free(sh[t].off); free(sh[t].pool.v); }
    free(sh);
    sh = NULL;
    if (rc) goto fin;
  }

  /* stage: group by exact signature (sort by signature, then fault order) */
  {
    int64_t *ord = (int64_t *)malloc((size_t)(nf ? nf : 1) * sizeof(int64_t));
    if (!ord) { rc = fail(ORC_E_OOM, "out of memory"); goto fin; }
    for (int64_t i = 0; i < nf; i++) ord[i] = i;
    sigctx_t g = {foff, pool.v};
    qsort_r(ord, (size_t)nf, sizeof(int64_t), cmp_fault, &g);
    res->edge_off = (int64_t *)malloc((size_t)(nf + 1) * sizeof(int64_t));
    res->edge_q = (double *)malloc((size_t)(nf ? nf : 1) * sizeof(double));
    res->edge_bits = (int32_t *)malloc((size_t)(pool.n ? pool.n : 1) * sizeof(int32_t));
    if (!res->edge_off || !res->edge_q || !res->edge_bits) { free(ord); rc = fail(ORC_E_OOM, "out of memory"); goto fin; }
    int64_t ne = 0, nb = 0;
    res->edge_off[0] = 0;
    int64_t i = 0;
    while (i < nf) {
      int64_t j = i + 1;
      int64_t li = foff[ord[i] + 1] - foff[ord[i]];
      while (j < nf) {
        int64_t lj = foff[ord[j] + 1] - foff[ord[j]];
        if (lj != li || memcmp(pool.v + foff[ord[i]], pool.v + foff[ord[j]], (size_t)li * sizeof(int32_t)))
          break;
        j++;
      }
      if (li == 0) {
        res->n_empty += j - i;
      } else {
        /* Eq. 3, merged in fault order */
        double q = 0.0;
        for (int64_t k = i; k < j; k++) {
          double p = fp[ord[k]];
          q = q * (1.0 - p) + p * (1.0 - q);
        }
        memcpy(res->edge_bits + nb, pool.v + foff[ord[i]], (size_t)li * sizeof(int32_t));
        nb += li;
        res->edge_q[ne] = q;
        res->edge_off[++ne] = nb;
      }
      i = j;
    }
    free(ord);
    res->n_edges = ne;
    res->n_edge_bits = nb;
  }
  res->n_qubits = c.nq;
  res->n_measurements = c.nmeas;
  res->n_detectors = c.ndet;
  res->n_observables = c.nobs;
  res->n_channels = c.nch;
  res->n_faults = nf;
  if (keep_faults) {
    res->fault_off = foff; foff = NULL;
    res->fault_bits = pool.v; pool.v = NULL;
    res->fault_p = fp; fp = NULL;
    res->fault_channel = fch; fch = NULL;
    res->fault_code = fcode; fcode = NULL;
  }
fin:
  free(foff); free(fp); free(fch); free(fch64); free(fcode);
  free(pool.v);
  free(sh);
  circ_free(&c);
  if (rc) { oracle_free(res); return rc; }
  *out = res;
  return ORC_OK;
}

/* --------------------------------------------------------------- gradient */

/* Derivative of the per-fault probability with respect to the channel rate,
 * from the split above: (1-2p)^k = 1 - x with x = a r gives
 * dp/dr = (a / (2k)) (1 - x)^(1/k - 1): DEPOLARIZE1 (k = 2, a = 4/3):
 * (1/3)(1 - 4r/3)^(-1/2); DEPOLARIZE2 (k = 8, a = 16/15):
 * (1/15)(1 - 16r/15)^(-7/8); a Pauli flip channel: 1. */
static double fault_dp_dr(int kind, double r) {
  switch (kind) {
    case N_DEP1: return (1.0 / 3.0) / sqrt(1.0 - 4.0 * r / 3.0);
    case N_DEP2: return (1.0 / 15.0) * pow(1.0 - 16.0 * r / 15.0, -7.0 / 8.0);
    default: return 1.0;
  }
}

/*
 * oracle_gradient: dL/d(rate) of every channel (program order) for a loss
 * whose derivative with respect to each hyperedge probability is given:
 * dl_dq[e] for the hyperedges in the order oracle_run returns them. With
 * q = 1/2 (1 - prod_j (1 - 2 p_j)) over the class members (Eq. 3 unrolled),
 * dq/dp_i = prod_{j != i} (1 - 2 p_j), evaluated here as that explicit
 * product; the chain rule then goes through dp_i/dr of the fault's channel.
 * Faults with an empty signature do not contribute.
 */
int oracle_gradient(const char *text, size_t len, const double *rates, int64_t n_rates, const double *dl_dq,
                    int64_t n_edges, double *dl_dr, int64_t n_out) {
  oracle_result *r = NULL;
  int rc = oracle_run(text, len, rates, n_rates, 1, 1, &r);
  if (rc) return rc;
  if (n_edges != r->n_edges) {
    int64_t ne = r->n_edges;
    oracle_free(r);
    return fail(ORC_E_ARG, "dl_dq has %lld entries, the hypergraph has %lld edges", (long long)n_edges,
                (long long)ne);
  }
  if (n_out != r->n_channels) {
    int64_t nc = r->n_channels;
    oracle_free(r);
    return fail(ORC_E_ARG, "dl_dr has %lld entries, the circuit has %lld channels", (long long)n_out, (long long)nc);
  }
  /* the channels' kinds and rates, as the forward pass used them */
  circ_t c;
  memset(&c, 0, sizeof c);
  if ((rc = parse(text, len, &c))) { oracle_free(r); circ_free(&c); return rc; }
  if (rates)
    for (int64_t k = 0; k < c.nch; k++) c.ch[k].rate = rates[k];
  for (int64_t k = 0; k < n_out; k++) dl_dr[k] = 0.0;
  const int64_t nf = r->n_faults;
  int64_t *ord = (int64_t *)malloc((size_t)(nf ? nf : 1) * sizeof(int64_t));
  if (!ord) { oracle_free(r); circ_free(&c); return fail(ORC_E_OOM, "out of memory"); }
  for (int64_t i = 0; i < nf; i++) ord[i] = i;
  sigctx_t g = {r->fault_off, r->fault_bits};
  qsort_r(ord, (size_t)nf, sizeof(int64_t), cmp_fault, &g);
  /* walk the classes in the order oracle_run emitted them */
  int64_t e = 0, i = 0;
  while (i < nf) {
    int64_t j = i + 1;
    const int64_t li = r->fault_off[ord[i] + 1] - r->fault_off[ord[i]];
    while (j < nf) {
      const int64_t lj = r->fault_off[ord[j] + 1] - r->fault_off[ord[j]];
      if (lj != li || memcmp(r->fault_bits + r->fault_off[ord[i]], r->fault_bits + r->fault_off[ord[j]],
                             (size_t)li * sizeof(int32_t)))
        break;
      j++;
    }
    if (li != 0) {
      for (int64_t a = i; a < j; a++) {
        double prod = 1.0;
        for (int64_t b = i; b < j; b++)
          if (b != a) prod *= 1.0 - 2.0 * r->fault_p[ord[b]];
        const int32_t ch = r->fault_channel[ord[a]];
        dl_dr[ch] += dl_dq[e] * prod * fault_dp_dr(c.ch[ch].kind, c.ch[ch].rate);
      }
      e++;
    }
    i = j;
  }
  free(ord);
  oracle_free(r);
  circ_free(&c);
  return ORC_OK;
}

/* Correlation level used by the following oracle_run / oracle_gradient calls
 * (0, 1 or 2 = every Pauli). */
int oracle_set_level(int level) {
  if (level < 0 || level > 2) return fail(ORC_E_ARG, "correlation level must be 0, 1 or 2");
  g_level = level;
  return ORC_OK;
}

/* Per-fault probability for a channel kind name, exposed so tests can pin the
 * split against closed forms. kind: 1 X_ERROR, 2 Y_ERROR, 3 Z_ERROR,
 * 4 DEPOLARIZE1, 5 DEPOLARIZE2. */
double oracle_fault_probability(int kind, double rate) { return fault_p(kind, rate); }
