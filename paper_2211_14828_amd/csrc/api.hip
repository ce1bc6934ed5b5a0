// C-ABI entry points (include/rbkitk.h) and the host-side driver of the
// hot path: per-mode rBKI (Alg. 1 and Alg. 2, steps 2-5), the core by a
// chain of mode products (Alg. 2, step 6), the explicit reconstruction error,
// and the TR-SVD branch of Alg. 3.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rbki_kernels.h"
#include "rbki_api_internal.h"

namespace rbki {
hipError_t tr_svd_device(const void* Gcore, int core_elem, int N, const int64_t* S, const int64_t* r,
                         double* const* cores, double* work, size_t work_bytes, int* info, double* discarded,
                         hipStream_t st);
size_t tr_svd_work_bytes(int N, const int64_t* S, const int64_t* r);
hipError_t tr_attach(const double* core, const double* Ut, int64_t ra, int64_t Sn, int64_t rb, int64_t I,
                     void* out, int out_elem, hipStream_t st);
hipError_t tr_gap2(const void* Gcore, int core_elem, int N, const int64_t* S, const int64_t* r,
                   double* const* cores, double* work, double* out, hipStream_t st);
size_t tr_gap2_work_bytes(int N, const int64_t* S, const int64_t* r);
size_t tr_als_work_bytes(int N, const int64_t* S, const int64_t* r);
hipError_t tr_als_device(const double* Gd, int N, const int64_t* S, const int64_t* r, double* const* cores,
                         uint64_t seed, int max_sweeps, double fit_tol, void* work, int* info, int* sweeps_out,
                         double* err2_out, hipStream_t st);
}  // namespace rbki

using namespace rbki;

namespace {

thread_local std::string g_err;

rbki_status fail(rbki_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                            \
  do {                                                                                          \
    hipError_t e__ = (expr);                                                                    \
    if (e__ != hipSuccess) return fail(RBKI_E_HIP, "%s: %s", #expr, hipGetErrorString(e__));    \
  } while (0)

// ------------------------------------------------------------------ timing
struct ProfRec {
  int64_t launches = 0;
  double ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::map<std::string, ProfRec> g_prof;

struct ProfScope {
  hipEvent_t a = nullptr, b = nullptr;
  const char* name;
  hipStream_t s;
  ProfScope(const char* n, hipStream_t st) : name(n), s(st) {
    if (!g_prof_on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
    (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[name].pending.push_back({a, b});
  }
};

void prof_drain() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& kv : g_prof) {
    for (auto& ev : kv.second.pending) {
      (void)hipEventSynchronize(ev.second);
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) {
        kv.second.ms += ms;
        kv.second.launches += 1;
      }
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
    kv.second.pending.clear();
  }
}

int cu_count() {
  // thread-safe one-time initialisation (the request server plans from
  // several host threads)
  static const int cached = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      return n;
    return 256;
  }();
  return cached;
}

// ------------------------------------------------------------------ planning
struct ModeGeom {
  int64_t A, I, B, J, R, S, Sp;   // Sp = S * (q + 1): rows of the Krylov basis buffer
  int64_t m = 0;                  // columns the Krylov basis is built from (J, or the sample)
  bool sampled = false;           // m < J: partial columns (Sec. 3.1)
  int yelem = 0;                  // element type of the gathered sample
  bool pipe = false;              // mixed forms: the pipelined Gram kernel on a blocked copy
  int pelem = 0;                  // its element type (E_BF16 or E_FP8)
  int64_t nkt = 0;                // its K tiles
};

struct Plan {
  int N = 0;
  int64_t dims[8], ranks[8];
  int p = 0, q = 0;
  uint64_t seed = 0;
  int prec = 0;
  int xelem = 0;     // storage of X
  int gelem = 0;     // Gram / sketch product
  int telem = 0;     // first mode product (reads X)
  int celem = 0;     // later mode products, reconstruction and error
  bool need_pad = false;     // mixed forms: zero-padded bf16 copy Xpad (first mode product, Gram fallback)
  bool need_xt16 = false;    // zero-padded bf16 transposed copy Xt (last mode on the Gram fallback)
  bool need_fp8 = false;     // e4m3 blocked copies with per-32 scales (fp8 Gram products)
  bool lead_pipe = false;    // some leading mode is pipelined: the one-pass blocked copy also writes Xpad
  bool first_blocked = false;   // the first mode product reads that mode's blocked copy
  bool need_xpad = false;    // some reader of Xpad remains (a Gram fallback or the first product)
  bool concurrent = false;   // runs beside other solves on the device (request server)
  bool power = false;        // power iteration: only the last block spans the factor's space
  double rate = 1.0;         // column sampling rate omega (Sec. 3.1)
  bool sequential = false;   // sequential truncation (ST-HOSVD form)
  bool one_stream = false;   // every mode on the caller's stream (no helper streams)
  bool fused = false;        // every mode's Krylov chain in one persistent launch (small modes)
  bool any_sampled = false;
  int64_t maxM = 0;          // largest column sample
  size_t ybytes = 0;         // largest gathered sample
  int64_t oblk_bytes = 0;                   // one mode's blocked bf16 sketch (the largest)
  int64_t in_pad = 0;        // last dimension padded to a multiple of 64
  int64_t rows_pad = 0;      // T / I_N padded to a multiple of 64 (row length of Xt)
  int64_t T = 1;
  ModeGeom m[8];
  int first_mode = 0;
  int64_t maxI = 0, maxS = 0, maxSp = 0, maxRI = 0, maxSJ = 0;
  size_t partial_bytes = 0;
  int64_t chain_elems = 0;   // largest intermediate of the core / reconstruction chains
};

int dtype_elem(int dt) { return dt == RBKI_F64 ? E_F64 : dt == RBKI_F32 ? E_F32 : E_BF16; }

// Mode n of the zero-padded operands: modes before the last read Xpad (or
// their blocked copy) as [A_n, I_n, Bp_n] with Bp_n = (B_n / I_N) I_Npad.
// The last mode reads Xt as [1, I_N, rows_pad], or its blocked copy as
// [1, I_N, H pad64(I_{N-1})] (H = T / (I_{N-1} I_N)): K runs over the rows of
// X with every run of I_{N-1} padded, so that a K tile stays inside one run.
void padded_view(const Plan& P, int n, bool pipe, int64_t& A, int64_t& Bp) {
  const ModeGeom& g = P.m[n];
  if (n == P.N - 1) {
    const int64_t L = P.dims[P.N - 2];
    A = 1;
    Bp = pipe ? (P.T / (L * P.dims[P.N - 1])) * pad64(L) : P.rows_pad;
  } else {
    A = g.A;
    Bp = (g.B / P.dims[P.N - 1]) * P.in_pad;
  }
}

// The sketch columns of mode n's blocked operand run as [A, B / IN, pad64(IN)]
// for these (B, IN): the view of padded_view.
void sketch_runs(const Plan& P, int n, int64_t& B, int64_t& IN) {
  const ModeGeom& g = P.m[n];
  if (n == P.N - 1) {
    B = g.J;
    IN = P.dims[P.N - 2];
  } else {
    B = g.B;
    IN = P.dims[P.N - 1];
  }
}

rbki_status make_plan(const rbki_params* prm, int xtype, Plan& P) {
  if (!prm) return fail(RBKI_E_INVALID, "params is NULL");
  if (prm->order < 2 || prm->order > 8) return fail(RBKI_E_INVALID, "order %d outside [2, 8]", prm->order);
  if (!prm->dims || !prm->ranks) return fail(RBKI_E_INVALID, "dims/ranks is NULL");
  if (xtype != RBKI_F64 && xtype != RBKI_F32 && xtype != RBKI_BF16)
    return fail(RBKI_E_INVALID, "unknown tensor dtype %d", xtype);
  if (prm->oversample < 0 || prm->power < 0 || prm->power > 64)
    return fail(RBKI_E_INVALID, "oversample %d / power %d out of range", prm->oversample, prm->power);
  if (prm->precision != RBKI_PLAIN && prm->precision != RBKI_MIXED_BF16 && prm->precision != RBKI_MIXED_FP8)
    return fail(RBKI_E_INVALID, "unknown precision %d", prm->precision);
  if (prm->variant != RBKI_KRYLOV && prm->variant != RBKI_POWER)
    return fail(RBKI_E_INVALID, "unknown variant %d", prm->variant);
  P.power = prm->variant == RBKI_POWER;
  if (prm->truncation != RBKI_INDEPENDENT && prm->truncation != RBKI_SEQUENTIAL)
    return fail(RBKI_E_INVALID, "unknown truncation %d", prm->truncation);
  P.sequential = prm->truncation == RBKI_SEQUENTIAL;
  {
    const double rate = prm->sample_rate == 0.0 ? 1.0 : prm->sample_rate;
    if (!(rate > 0.0 && rate <= 1.0))
      return fail(RBKI_E_INVALID, "sample_rate %g outside (0, 1]", prm->sample_rate);
    P.rate = rate;
  }
  P.N = prm->order;
  P.p = prm->oversample;
  P.q = prm->power;
  P.seed = prm->seed;
  P.prec = prm->precision;
  P.T = 1;
  for (int n = 0; n < P.N; ++n) {
    P.dims[n] = prm->dims[n];
    P.ranks[n] = prm->ranks[n];
    if (P.dims[n] < 1) return fail(RBKI_E_INVALID, "dims[%d] = %lld < 1", n, (long long)P.dims[n]);
    P.T *= P.dims[n];
  }
  P.xelem = dtype_elem(xtype);
  // the first mode product always reads X itself, in its own type
  P.telem = P.xelem;
  P.gelem = P.prec == RBKI_PLAIN ? P.xelem : (P.prec == RBKI_MIXED_FP8 ? E_FP8 : E_BF16);
  P.need_pad = P.gelem == E_BF16 || P.gelem == E_FP8;
  P.need_fp8 = P.gelem == E_FP8;
  // chain and error in float64 only for the plain float64 form (the bf16
  // forms' first product writes float)
  P.celem = (P.xelem == E_F64 && !P.need_pad) ? E_F64 : E_F32;
  P.in_pad = pad64(P.dims[P.N - 1]);
  P.rows_pad = pad64(P.T / P.dims[P.N - 1]);
  double best = -1.0;
  for (int n = 0; n < P.N; ++n) {
    ModeGeom& g = P.m[n];
    g.A = 1;
    for (int k = 0; k < n; ++k) g.A *= P.dims[k];
    g.I = P.dims[n];
    g.B = 1;
    for (int k = n + 1; k < P.N; ++k) g.B *= P.dims[k];
    g.J = g.A * g.B;
    g.R = P.ranks[n];
    if (g.R < 1 || g.R > g.I || g.R > g.J)
      return fail(RBKI_E_INVALID, "ranks[%d] = %lld outside [1, min(I_n, J_n)]", n, (long long)g.R);
    g.m = sample_count(g.J, P.rate);
    g.sampled = g.m < g.J;
    if (g.m < g.R)
      return fail(RBKI_E_INVALID, "sample_rate %g leaves %lld columns in mode %d, fewer than its rank %lld",
                  P.rate, (long long)g.m, n, (long long)g.R);
    g.S = std::min<int64_t>(std::min<int64_t>(g.R + P.p, g.I), g.m);   // Sec. 2.3, Sec. 4.1
    g.Sp = P.power ? g.S : g.S * (P.q + 1);
    if (g.Sp > 1200) return fail(RBKI_E_UNSUPPORTED, "Krylov width %lld > 1200 (mode %d)", (long long)g.Sp, n);
    const double ratio = (double)g.I / (double)g.R;
    if (ratio > best) { best = ratio; P.first_mode = n; }
    P.maxI = std::max(P.maxI, g.I);
    P.maxS = std::max(P.maxS, g.S);
    P.maxSp = std::max(P.maxSp, g.Sp);
    P.maxRI = std::max(P.maxRI, g.R * g.I);
    if (g.sampled) {
      // the Krylov products read the gathered sample (bf16 in the mixed forms)
      g.yelem = P.need_pad ? E_BF16 : P.xelem;
      P.any_sampled = true;
      P.maxM = std::max(P.maxM, g.m);
      P.ybytes = std::max(P.ybytes, (size_t)g.I * g.m * elem_size(g.yelem));
      P.maxSJ = std::max(P.maxSJ, g.S * g.m);
      GramArgs gy = gram_plan(g.yelem, 1, g.I, g.m, (int)g.S, cu_count());
      P.partial_bytes = std::max(P.partial_bytes, gram_partial_bytes(gy, g.yelem));
    }
    if (P.need_pad) {
      int64_t A, Bp;
      g.pipe = gram_pipe_ok(g.I, (int)g.S);
      padded_view(P, n, g.pipe, A, Bp);
      if (g.pipe) {
        g.pelem = P.need_fp8 ? E_FP8 : E_BF16;
        const int64_t KT = g.pelem == E_FP8 ? 64 : 32;
        g.nkt = A * Bp / KT;
        P.oblk_bytes = std::max(P.oblk_bytes, g.nkt * 64 * KT * 2);
        P.partial_bytes = std::max(P.partial_bytes,
                                   gram_pipe_partial_bytes(gram_plan_pipe(g.pelem, A, g.I, Bp, (int)g.S, cu_count())));
      } else {
        P.maxSJ = std::max(P.maxSJ, g.S * A * Bp);
        if (n == P.N - 1) P.need_xt16 = true;
        GramArgs ga = gram_plan(E_BF16, A, g.I, Bp, (int)g.S, cu_count());
        P.partial_bytes = std::max(P.partial_bytes, gram_partial_bytes(ga, E_BF16));
      }
    } else {
      P.maxSJ = std::max(P.maxSJ, g.S * g.J);
      GramArgs ga = gram_plan(P.gelem, g.A, g.I, g.B, (int)g.S, cu_count());
      P.partial_bytes = std::max(P.partial_bytes, gram_partial_bytes(ga, P.gelem));
    }
  }
  if (P.need_pad) {
    bool fallback_lead = false;
    for (int n = 0; n + 1 < P.N; ++n) {
      P.lead_pipe = P.lead_pipe || P.m[n].pipe;
      fallback_lead = fallback_lead || !P.m[n].pipe;
    }
    const ModeGeom& gf = P.m[P.first_mode];
    P.first_blocked = P.first_mode < P.N - 1 && gf.pipe && gf.R <= 64;
    P.need_xpad = fallback_lead || !P.first_blocked;
  }
  // chain sizes: core chain starting with first_mode, then ascending; the
  // reconstruction chain expands modes 1..N-1 from the core.
  int64_t cur[8];
  for (int n = 0; n < P.N; ++n) cur[n] = P.dims[n];
  int64_t mx = 0;
  auto prod = [&](const int64_t* d) { int64_t t = 1; for (int k = 0; k < P.N; ++k) t *= d[k]; return t; };
  cur[P.first_mode] = P.ranks[P.first_mode];
  mx = std::max(mx, prod(cur));
  for (int n = 0; n < P.N; ++n)
    if (n != P.first_mode) { cur[n] = P.ranks[n]; mx = std::max(mx, prod(cur)); }
  for (int n = 1; n < P.N; ++n) { cur[n] = P.dims[n]; mx = std::max(mx, prod(cur)); }
  P.chain_elems = mx;
  // small modes: the Krylov chains (Alg. 1 after the Gram pass, and Z) of
  // all modes in one launch, one workgroup per mode
  P.fused = !P.any_sampled;
  for (int n = 0; n < P.N; ++n) P.fused = P.fused && krylov_chain_ok(P.m[n].I, P.m[n].S);
  return RBKI_OK;
}

constexpr size_t kDgemmScratch = (size_t)32 << 20;

struct Arena {
  char* base;
  size_t off = 0, cap;
  bool sizing;
  Arena(void* b, size_t c) : base((char*)b), cap(c), sizing(b == nullptr) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = sizing ? nullptr : base + off;
    off += bytes;
    return p;
  }
};

// Scratch of one mode's sketch, Gram and Krylov steps.  Large problems get
// one set per concurrently running mode (see mode_lanes).
struct Lane {
  void* oblk = nullptr;    // the mode's blocked sketch: bf16, then e4m3 + scales
  void* om8 = nullptr;
  void* oscl = nullptr;
  void* omegaT = nullptr;
  void* partial = nullptr;
  double* C = nullptr;
  double* CQt = nullptr;
  double* Yt = nullptr;
  double* Ytmp = nullptr;
  double* Pm = nullptr;
  double* dscratch = nullptr;   // split-K partials of the float64 GEMMs
  double* G = nullptr;
  double* L = nullptr;
  int* flags = nullptr;
  double* ref2 = nullptr;
  double* CY = nullptr;     // partial columns: Y Y^T of the sample
  void* ysmp = nullptr;     //   the gathered sample Y (I x m)
  int64_t* cols = nullptr;  //   its column indices
};
constexpr int kMaxLanes = 3;

struct Buffers {
  void* xpad = nullptr;    // bf16, (T / I_N) x I_Npad, zero-padded
  void* xb[8] = {};        // each pipelined mode's blocked copy (bf16 or e4m3) and its e4m3 scales
  void* xs[8] = {};
  void* xt = nullptr;      // bf16, I_N x rows_pad: the last mode, transposed and zero-padded
  void* u16 = nullptr;     // the first product's factor as bf16 [64][block rows]
  Lane ln[8];
  int lanes = 1;             // scratch sets of concurrently running modes
  int chain_lanes = 1;       // scratch sets of the Krylov chains (one per mode in a fused plan)
  double* Qt[8] = {};      // per mode: S'_n x I_n basis rows
  double* Z[8] = {};       // per mode: S'_n x S'_n
  double* lam[8] = {};
  double* Vt[8] = {};
  void* jwork[8] = {};
  int* info = nullptr;
  int* used = nullptr;       // per mode, q + 2 slots: directions kept by blocks 0..j-1
  double* Ut64[8] = {};
  void* Uop = nullptr;     // one factor in a product element type
  void* chainA = nullptr;
  void* chainB = nullptr;
  void* gkeep = nullptr;   // the core, kept apart from the reconstruction chain
  void* rpartial = nullptr;
  double* sums = nullptr;
};

// Modes whose sketch, Gram and Krylov steps may run at the same time on
// their own streams: on large tensors the Krylov steps are chains of small
// latency-bound kernels that overlap well with each other and with the next
// mode's Gram kernel.  Fixed by the problem alone, so that the workspace is
// the same for every caller.
int mode_lanes(const Plan& P) { return (P.T >= ((int64_t)1 << 26) && P.N > 1) ? std::min(P.N, kMaxLanes) : 1; }

// Jacobi info (2 ints per mode) and the per-mode direction counts, zeroed
// together before a decomposition.
size_t counters_bytes(const Plan& P) { return 256 + (size_t)P.N * (P.q + 2) * 4; }

void carve(const Plan& P, Arena& ar, Buffers& b) {
  const int es_g = elem_size(P.gelem);
  if (P.need_pad) {
    const size_t rows = (size_t)(P.T / P.dims[P.N - 1]);
    if (P.need_xpad) b.xpad = ar.take(rows * P.in_pad * 2);
    if (P.first_blocked) b.u16 = ar.take((size_t)64 * block_rows(P.m[P.first_mode].I) * 2);
    if (P.need_xt16) b.xt = ar.take((size_t)P.dims[P.N - 1] * P.rows_pad * 2);
    for (int n = 0; n < P.N; ++n) {
      const ModeGeom& g = P.m[n];
      if (!g.pipe) continue;
      b.xb[n] = ar.take(block_copy_bytes(g.nkt, g.I));
      if (g.pelem == E_FP8) b.xs[n] = ar.take((size_t)g.nkt * block_rows(g.I) * 2);
    }
  }
  b.lanes = mode_lanes(P);
  b.chain_lanes = P.fused ? std::max(b.lanes, P.N) : b.lanes;
  for (int l = 0; l < b.chain_lanes; ++l) {
    Lane& L = b.ln[l];
    if (l >= b.lanes) {
      // a fused plan's extra sets: chain buffers of their own; the sketch and
      // Gram scratch of set 0 (those passes run one after the other)
      L = b.ln[0];
      L.C = (double*)ar.take((size_t)P.maxI * P.maxI * 8);
      L.CQt = (double*)ar.take((size_t)P.maxSp * P.maxI * 8);
      L.Yt = (double*)ar.take((size_t)P.maxS * P.maxI * 8);
      L.Ytmp = (double*)ar.take((size_t)P.maxS * P.maxI * 8);
      L.Pm = (double*)ar.take((size_t)P.maxS * P.maxSp * 8);
      L.G = (double*)ar.take((size_t)P.maxS * P.maxS * 8);
      continue;
    }
    if (P.need_pad && P.oblk_bytes) {
      if (!P.need_fp8) L.oblk = ar.take((size_t)P.oblk_bytes);   // the fp8 sketch is made in one pass
      if (P.need_fp8) {
        L.om8 = ar.take((size_t)P.oblk_bytes / 2);
        L.oscl = ar.take((size_t)P.oblk_bytes / 32 + 256);    // 256 bytes per K tile
      }
    }
    L.omegaT = ar.take((size_t)P.maxSJ * (P.need_pad ? 2 : es_g));   // the fallback of the mixed forms: bf16
    L.partial = ar.take(P.partial_bytes);
    L.C = (double*)ar.take((size_t)P.maxI * P.maxI * 8);
    L.CQt = (double*)ar.take((size_t)P.maxSp * P.maxI * 8);
    L.Yt = (double*)ar.take((size_t)P.maxS * P.maxI * 8);
    L.Ytmp = (double*)ar.take((size_t)P.maxS * P.maxI * 8);
    L.Pm = (double*)ar.take((size_t)P.maxS * P.maxSp * 8);
    L.dscratch = (double*)ar.take(kDgemmScratch);
    L.G = (double*)ar.take((size_t)P.maxS * P.maxS * 8);
    L.L = (double*)ar.take((size_t)P.maxS * P.maxS * 8);
    L.flags = (int*)ar.take((size_t)P.maxSp * 4);
    L.ref2 = (double*)ar.take((size_t)P.maxS * 8);
    if (P.any_sampled) {
      L.CY = (double*)ar.take((size_t)P.maxI * P.maxI * 8);
      L.ysmp = ar.take(P.ybytes);
      L.cols = (int64_t*)ar.take((size_t)P.maxM * 8);
    }
  }
  for (int n = 0; n < P.N; ++n) b.Qt[n] = (double*)ar.take((size_t)P.m[n].Sp * P.m[n].I * 8);
  for (int n = 0; n < P.N; ++n) {
    const int64_t Sp = P.m[n].Sp;
    b.Z[n] = (double*)ar.take((size_t)Sp * Sp * 8);
    b.lam[n] = (double*)ar.take((size_t)Sp * 8);
    b.Vt[n] = (double*)ar.take((size_t)Sp * Sp * 8);
    const int64_t R = P.m[n].R;
    // the leading-eigenpair solver takes Z up to 512 wide (also the narrower
    // Z of the first steps of an adaptive solve)
    const int64_t et = std::min<int64_t>(Sp, 512);
    b.jwork[n] = ar.take(std::max(jacobi_work_bytes(Sp), eig_top_ok(et, R) ? eig_top_work_bytes(et, R) : (size_t)0));
  }
  b.info = (int*)ar.take(counters_bytes(P));
  b.used = b.info + 64;
  for (int n = 0; n < P.N; ++n) b.Ut64[n] = (double*)ar.take((size_t)P.m[n].R * P.m[n].I * 8);
  b.Uop = ar.take((size_t)P.maxRI * 8);
  const size_t ce = P.celem == E_F64 ? 8 : 4;
  b.chainA = ar.take((size_t)P.chain_elems * ce);
  b.chainB = ar.take((size_t)P.chain_elems * ce);
  int64_t ncore = 1;
  for (int n = 0; n < P.N; ++n) ncore *= P.ranks[n];
  b.gkeep = ar.take((size_t)ncore * ce);
  b.rpartial = ar.take(residual_work_bytes(P.dims[0], P.T / P.dims[0]));
  b.sums = (double*)ar.take(64);
}

size_t plan_bytes(const Plan& P) {
  Arena ar(nullptr, 0);
  Buffers b;
  carve(P, ar, b);
  return ar.off + 256;
}

// The copies of X the mixed forms read, made once per decomposition: the
// blocked copies of every pipelined mode in one pass over X (which also
// writes the padded bf16 copy Xpad where something reads it), and Xpad / Xt
// by the plain padding pass where no blocked pass writes them.
rbki_status convert_input(const Plan& P, const Buffers& b, const void* X, hipStream_t st) {
  const int64_t IN = P.dims[P.N - 1];
  const bool any_pipe = P.lead_pipe || P.m[P.N - 1].pipe;
  if (any_pipe) {
    bool want[8] = {};
    void* outs[8] = {};
    void* scs[8] = {};
    for (int n = 0; n < P.N; ++n) {
      want[n] = P.m[n].pipe;
      outs[n] = b.xb[n];
      scs[n] = b.xs[n];
    }
    HIPCHK(launch_block_copies(P.xelem, P.need_fp8 ? E_FP8 : E_BF16, X, P.N, P.dims, want, outs, scs,
                               (P.lead_pipe && P.need_xpad) ? b.xpad : nullptr, st));
  }
  if (!P.lead_pipe || P.need_xt16)
    HIPCHK(launch_pad_copies(P.xelem, X, P.T / IN, IN, P.lead_pipe ? nullptr : b.xpad, b.xt, st));
  return RBKI_OK;
}

// ------------------------------------------------------------------ one mode
// Alg. 1 + Alg. 2 steps 1-3 for mode n, in two parts: run_mode_heavy (the
// sketch and the Gram / sketch products, C and W into the scratch set) and
// run_mode_chain (the Krylov basis in b.Qt, Sp rows, C Q in the set's CQt,
// and Z).
constexpr double TAU_REL = 1e-12;   // pivot vs its own column: direction already spanned
constexpr double TAU_ABS = 1e-10;   // pivot vs the block before projection (matches the oracle)

// heavy_wait / heavy_done (nullable): events that the sketch and Gram
// kernels wait for and record, so that those throughput-bound kernels of
// concurrently running modes follow each other.
rbki_status run_mode_heavy(const Plan& P, const Buffers& b, int lane, const void* xsrc, int n, hipStream_t st,
                           hipEvent_t heavy_wait = nullptr, hipEvent_t heavy_done = nullptr) {
  const Lane& L = b.ln[lane];
  dgemm_set_scratch(L.dscratch, kDgemmScratch);
  if (heavy_wait) HIPCHK(hipStreamWaitEvent(st, heavy_wait, 0));
  const ModeGeom& g = P.m[n];
  const int64_t I = g.I, S = g.S;
  // C -> L.C (I x I), W^T -> L.Yt (S x I)
  if (P.need_pad) {
    int64_t A, Bp;
    padded_view(P, n, g.pipe, A, Bp);
    const bool last = n == P.N - 1;
    if (g.pipe) {
      // the blocked copy of this mode's unfolding was made by convert_input;
      // the blocked sketch
      const int KT = g.pelem == E_FP8 ? 64 : 32;
      int64_t SB, SIN;
      sketch_runs(P, n, SB, SIN);
      {
        ProfScope ps("omega", st);
        if (g.pelem == E_FP8) {
          HIPCHK(launch_omega_fp8(P.seed, n, S, g.J, SB, SIN, g.nkt, L.om8, L.oscl, st));
        } else {
          HIPCHK(launch_omega_block(P.seed, n, S, g.J, SB, SIN, g.nkt, KT, L.oblk, st));
        }
      }
      GramArgs ga = gram_plan_pipe(g.pelem, A, I, Bp, (int)S, cu_count());
      ga.X = b.xb[n];
      ga.omegaT = g.pelem == E_FP8 ? L.om8 : L.oblk;
      ga.xexp = (const unsigned char*)b.xs[n];
      ga.xexp_om = (const unsigned char*)L.oscl;
      ga.partial = L.partial;
      {
        ProfScope ps("gram", st);
        HIPCHK(launch_gram_pipe(g.pelem, ga, st));
      }
      HIPCHK(launch_gram_pipe_reduce(ga, L.C, L.Yt, st));
    } else {
      // small I or a sketch wider than 64: the bf16 kernel on the padded copies
      {
        ProfScope ps("omega", st);
        HIPCHK(launch_omega_pad(P.seed, n, S, g.J, g.B, P.dims[P.N - 1], A * Bp, L.omegaT, st));
      }
      GramArgs ga = gram_plan(E_BF16, A, I, Bp, (int)S, cu_count());
      ga.X = last ? b.xt : b.xpad;
      ga.omegaT = L.omegaT;
      ga.partial = L.partial;
      {
        ProfScope ps("gram", st);
        HIPCHK(launch_gram_main(E_BF16, ga, st));
      }
      HIPCHK(launch_gram_reduce(E_BF16, ga, L.C, L.Yt, st));
    }
  } else {
    // a sampled mode needs only C from the whole unfolding (for Z): no sketch
    const int Sf = g.sampled ? 0 : (int)S;
    if (Sf) {
      ProfScope ps("omega", st);
      HIPCHK(launch_omega(P.gelem, P.seed, n, S * g.J, L.omegaT, st));
    }
    GramArgs ga = gram_plan(P.gelem, g.A, g.I, g.B, Sf, cu_count());
    ga.X = xsrc;
    ga.omegaT = L.omegaT;
    ga.partial = L.partial;
    {
      ProfScope ps("gram", st);
      HIPCHK(launch_gram_main(P.gelem, ga, st));
    }
    HIPCHK(launch_gram_reduce(P.gelem, ga, L.C, L.Yt, st));
  }

  if (g.sampled) {
    // Sec. 3.1, partial columns: the Krylov basis comes from the sampled
    // columns Y of the unfolding; C_Y = Y Y^T and W = Y Omega (Omega of m
    // rows) from the gathered sample
    HIPCHK(launch_sample_columns(P.seed, n, g.J, g.m, L.cols, st));
    HIPCHK(launch_gather_columns(P.xelem, xsrc, I, g.B, L.cols, g.m, g.yelem, L.ysmp, st));
    {
      ProfScope ps("omega", st);
      HIPCHK(launch_omega(g.yelem, P.seed, n, S * g.m, L.omegaT, st));
    }
    GramArgs gy = gram_plan(g.yelem, 1, I, g.m, (int)S, cu_count());
    gy.X = L.ysmp;
    gy.omegaT = L.omegaT;
    gy.partial = L.partial;
    {
      ProfScope ps("gram_sample", st);
      HIPCHK(launch_gram_main(g.yelem, gy, st));
    }
    HIPCHK(launch_gram_reduce(g.yelem, gy, L.CY, L.Yt, st));
  }

  if (heavy_done) HIPCHK(hipEventRecord(heavy_done, st));
  return RBKI_OK;
}

// Alg. 1, block 0: Q_0 = orth(W) from W^T in the lane's Yt.  The first pass
// of every block's CholeskyQR2 also keeps the basis at most I_n wide: once
// it spans the whole space the later blocks are rounding noise and are
// dropped whatever their norm.
rbki_status krylov_block0(const Plan& P, const Buffers& b, const Lane& L, int n, hipStream_t st) {
  const ModeGeom& g = P.m[n];
  const int64_t I = g.I, S = g.S;
  int* used = b.used + (size_t)n * (P.q + 2);
  HIPCHK(row_norms2(L.Yt, S, I, L.ref2, st));
  HIPCHK(chol_orth(L.Yt, L.Ytmp, S, I, L.G, L.L, L.flags, L.ref2, TAU_REL, TAU_ABS, st, DimBudget{used, used + 1, I}));
  HIPCHK(chol_orth(L.Ytmp, b.Qt[n], S, I, L.G, L.L, L.flags, nullptr, TAU_REL, 0.0, st));
  return RBKI_OK;
}

// Alg. 1, Krylov step j >= 1: block j of the basis from (X X^T) Q_{j-1} (Ck
// is X X^T, or Y Y^T of a sampled mode), projected off the earlier blocks
// twice and orthonormalised.  The product C Q_{j-1} is formed into the
// lane's Yt and, when CQ is given, kept as rows (j-1) S.. of CQ; with from_cq
// it is taken from there instead (formed earlier with the same C).
rbki_status krylov_step(const Plan& P, const Buffers& b, const Lane& L, int n, int j, const double* Ck, double* CQ,
                        bool from_cq, hipStream_t st) {
  const ModeGeom& g = P.m[n];
  const int64_t I = g.I, S = g.S;
  double* Qt = b.Qt[n];
  int* used = b.used + (size_t)n * (P.q + 2);
  const int64_t m = S * j;                     // rows of the basis so far
  const double* Qlast = Qt + (m - S) * I;
  if (from_cq) {
    HIPCHK(copy_rows_f64(L.Yt, I, CQ + (m - S) * I, I, S, I, st));
  } else {
    // Y_j^T = Q_{j-1}^T C  (C symmetric)
    HIPCHK(dgemm(0, 0, S, I, I, 1.0, Qlast, I, Ck, I, 0.0, L.Yt, I, st));
    if (CQ) HIPCHK(copy_rows_f64(CQ + (m - S) * I, I, L.Yt, I, S, I, st));
  }
  HIPCHK(row_norms2(L.Yt, S, I, L.ref2, st));
  for (int pass = 0; pass < 2; ++pass) {       // remove earlier blocks, twice
    HIPCHK(dgemm(0, 1, S, m, I, 1.0, L.Yt, I, Qt, I, 0.0, L.Pm, m, st));
    HIPCHK(dgemm(0, 0, S, I, m, -1.0, L.Pm, m, Qt, I, 1.0, L.Yt, I, st));
  }
  HIPCHK(chol_orth(L.Yt, L.Ytmp, S, I, L.G, L.L, L.flags, L.ref2, TAU_REL, TAU_ABS, st,
                   DimBudget{used + j, used + j + 1, I}));
  HIPCHK(chol_orth(L.Ytmp, Qt + m * I, S, I, L.G, L.L, L.flags, nullptr, TAU_REL, 0.0, st));
  return RBKI_OK;
}

// Alg. 2, steps 2-3 of mode n after run_mode_heavy: the Krylov basis from C
// and W in the scratch set, and Z.
rbki_status run_mode_chain(const Plan& P, const Buffers& b, int lane, int n, bool with_factor, hipStream_t st) {
  const Lane& L = b.ln[lane];
  dgemm_set_scratch(L.dscratch, kDgemmScratch);
  const ModeGeom& g = P.m[n];
  const int64_t I = g.I, S = g.S, Sp = g.Sp;
  double* Qt = b.Qt[n];
  // the Krylov products: with the sample's Y Y^T for a sampled mode
  const double* Ck = g.sampled ? L.CY : L.C;
  rbki_status s = krylov_block0(P, b, L, n, st);
  if (s != RBKI_OK) return s;
  if (P.power) {
    // power iteration (Sec. 3.1): Q_j = orth(C Q_{j-1}), each step's block
    // replacing the last, with the same drop rule relative to the step's
    // largest squared row norm
    for (int j = 1; j <= P.q; ++j) {
      HIPCHK(dgemm(0, 0, S, I, I, 1.0, Qt, I, Ck, I, 0.0, L.Yt, I, st));
      HIPCHK(row_norms2(L.Yt, S, I, L.ref2, st));
      HIPCHK(chol_orth(L.Yt, L.Ytmp, S, I, L.G, L.L, L.flags, L.ref2, TAU_REL, TAU_ABS, st));
      HIPCHK(chol_orth(L.Ytmp, Qt, S, I, L.G, L.L, L.flags, nullptr, TAU_REL, 0.0, st));
    }
    if (!with_factor) return RBKI_OK;
    HIPCHK(dgemm(0, 0, S, I, I, 1.0, Qt, I, L.C, I, 0.0, L.CQt, I, st));
    HIPCHK(dgemm(0, 1, S, S, I, 1.0, Qt, I, L.CQt, I, 0.0, b.Z[n], S, st));
    return RBKI_OK;
  }
  for (int j = 1; j <= P.q; ++j) {
    s = krylov_step(P, b, L, n, j, Ck, L.CQt, false, st);
    if (s != RBKI_OK) return s;
  }
  if (!with_factor) return RBKI_OK;
  // C Q_q, then Z = Q^T (C Q) (Alg. 2, step 3); a sampled mode's earlier
  // products were with Y Y^T, so C Q is formed for the whole basis
  if (g.sampled) {
    HIPCHK(dgemm(0, 0, Sp, I, I, 1.0, Qt, I, L.C, I, 0.0, L.CQt, I, st));
  } else {
    HIPCHK(dgemm(0, 0, S, I, I, 1.0, Qt + (Sp - S) * I, I, L.C, I, 0.0, L.CQt + (Sp - S) * I, I, st));
  }
  HIPCHK(dgemm(0, 1, Sp, Sp, I, 1.0, Qt, I, L.CQt, I, 0.0, b.Z[n], Sp, st));
  return RBKI_OK;
}

// The persistent chain of mode n on scratch set `lane` (fused plans): blocks
// j0..j1 of the basis, then Z over its first zr rows (zr = 0: no Z).
ChainJob chain_job(const Plan& P, const Buffers& b, int lane, int n, int zr) {
  const Lane& L = b.ln[lane];
  const ModeGeom& g = P.m[n];
  ChainJob j;
  j.C = L.C;
  j.Yt = L.Yt;
  j.Ytmp = L.Ytmp;
  j.Pm = L.Pm;
  j.G = L.G;
  j.CQ = L.CQt;
  j.Qt = b.Qt[n];
  j.Z = b.Z[n];
  j.used = b.used + (size_t)n * (P.q + 2);
  j.I = (int)g.I;
  j.S = (int)g.S;
  j.zr = zr;
  return j;
}

rbki_status run_chains(const Plan& P, const ChainJob* jobs, int njobs, int j0, int j1, hipStream_t st) {
  ChainArgs a = {};
  a.power = P.power ? 1 : 0;
  for (int i = 0; i < njobs; ++i) a.job[i] = jobs[i];
  a.j0 = j0;
  a.j1 = j1;
  a.tau_rel = TAU_REL;
  a.tau_abs = TAU_ABS;
  ProfScope ps("chain", st);
  HIPCHK(launch_krylov_chain(a, njobs, st));
  return RBKI_OK;
}

rbki_status run_mode(const Plan& P, const Buffers& b, int lane, const void* xsrc, int n, bool with_factor,
                     hipStream_t st) {
  rbki_status s = run_mode_heavy(P, b, lane, xsrc, n, st);
  if (s != RBKI_OK) return s;
  if (P.fused) {
    const ChainJob j = chain_job(P, b, lane, n, with_factor ? (int)P.m[n].Sp : 0);
    return run_chains(P, &j, 1, 0, P.q, st);
  }
  return run_mode_chain(P, b, lane, n, with_factor, st);
}

// Alg. 2, steps 4-5 for mode n alone, on stream st (the mode's stream when
// the modes run concurrently): its R leading eigenvectors (ordinary launch:
// the solve runs beside other modes' work) and U^T = Vt(1:R, :) Q^T with the
// sign rule.  For modes whose Z the leading-eigenpair solver takes.
rbki_status factor_one(const Plan& P, const Buffers& b, int n, hipStream_t st) {
  const ModeGeom& g = P.m[n];
  const double* Z = b.Z[n];
  int64_t sn = g.Sp, rn = g.R;
  double* lam = b.lam[n];
  double* Vt = b.Vt[n];
  void* w = b.jwork[n];
  int* info = b.info + 2 * n;
  {
    // the last mode's solve is the one the decomposition waits for
    ProfScope ps(n == P.N - 1 ? "eig" : "eig_early", st);
    HIPCHK(eig_top_batched(1, &Z, &sn, &rn, &lam, &Vt, &w, &info, st, false));
  }
  HIPCHK(dgemm(0, 0, g.R, g.I, g.Sp, 1.0, b.Vt[n], g.Sp, b.Qt[n], g.I, 0.0, b.Ut64[n], g.I, st));
  HIPCHK(canonical_sign_rows(b.Ut64[n], g.R, g.I, st));
  return RBKI_OK;
}

// Alg. 2, steps 4-5 for mode n alone, on the caller's stream (the stages of
// the sequential form): the R leading eigenpairs of Z (the Jacobi solver
// beyond that solver's sizes), U^T = Vt(1:R, :) Q^T, sign rule.
rbki_status factor_single(const Plan& P, const Buffers& b, int n, hipStream_t st, int64_t width = 0) {
  const ModeGeom& g = P.m[n];
  const double* Z = b.Z[n];
  int64_t sn = width > 0 ? width : g.Sp, rn = g.R;
  double* lam = b.lam[n];
  double* Vt = b.Vt[n];
  void* w = b.jwork[n];
  int* info = b.info + 2 * n;
  {
    ProfScope ps("eig", st);
    if (eig_top_ok(sn, rn)) {
      HIPCHK(eig_top_batched(1, &Z, &sn, &rn, &lam, &Vt, &w, &info, st, !P.concurrent));
    } else {
      HIPCHK(jacobi_eig_batched(1, &Z, &sn, &lam, &Vt, &w, &info, 40, st, P.concurrent && sn <= 192));
    }
  }
  HIPCHK(dgemm(0, 0, g.R, g.I, sn, 1.0, b.Vt[n], sn, b.Qt[n], g.I, 0.0, b.Ut64[n], g.I, st));
  HIPCHK(canonical_sign_rows(b.Ut64[n], g.R, g.I, st));
  return RBKI_OK;
}

// Alg. 2, steps 4-5 for all modes: the R leading eigenvectors of every Z in
// one launch (tridiagonal reduction, bisection, inverse iteration; block
// Jacobi for matrices beyond that solver's sizes), then U^T = Vt(1:R, :) Q^T
// with the sign rule.
rbki_status run_factors(const Plan& P, const Buffers& b, hipStream_t st) {
  const double* Zs[8];
  int64_t ns[8], rs[8];
  double* ls[8];
  double* vs[8];
  void* ws[8];
  int* is[8];
  bool top = true;
  for (int n = 0; n < P.N; ++n) {
    Zs[n] = b.Z[n];
    ns[n] = P.m[n].Sp;
    rs[n] = P.m[n].R;
    ls[n] = b.lam[n];
    vs[n] = b.Vt[n];
    ws[n] = b.jwork[n];
    is[n] = b.info + 2 * n;
    top = top && eig_top_ok(ns[n], rs[n]);
  }
  {
    ProfScope ps("eig", st);
    if (top) {
      // beside other solves (the request server) the multi-workgroup
      // reduction takes the ordinary launch: a cooperative grid does not
      // share the device with work on other streams
      HIPCHK(eig_top_batched(P.N, Zs, ns, rs, ls, vs, ws, is, st, !P.concurrent));
    } else {
      // beside other solves (the request server) small matrices take the
      // ordinary per-matrix launch: a cooperative grid does not share the
      // device with work on other streams
      int64_t nmax = 0;
      for (int n = 0; n < P.N; ++n) nmax = std::max(nmax, ns[n]);
      HIPCHK(jacobi_eig_batched(P.N, Zs, ns, ls, vs, ws, is, 40, st, P.concurrent && nmax <= 192));
    }
  }
  for (int n = 0; n < P.N; ++n) {
    const ModeGeom& g = P.m[n];
    HIPCHK(dgemm(0, 0, g.R, g.I, g.Sp, 1.0, b.Vt[n], g.Sp, b.Qt[n], g.I, 0.0, b.Ut64[n], g.I, st));
    // sign rule: largest-magnitude entry of each factor column positive
    HIPCHK(canonical_sign_rows(b.Ut64[n], g.R, g.I, st));
  }
  return RBKI_OK;
}

// Core chain and error.  Returns the core (chain element type) in *core_out.
// Alg. 2, step 6, first product: G_1 = X x_f U^(f)T for the first mode f of
// the core chain, into b.chainA.  It reads X (or the mode's blocked copy) and
// U^(f) only, so it may run as soon as that factor exists.
rbki_status first_product(const Plan& P, const Buffers& b, const void* xsrc, hipStream_t st) {
  const int n = P.first_mode;
  const int64_t A = P.m[n].A, I = P.m[n].I, B = P.m[n].B;
  void* out = b.chainA;
  if (P.first_blocked) {
    // precision form: the product reads the mode's blocked copy (the Gram
    // operand), decoded to bf16, on bf16 MFMA
    ProfScope ps("ttm", st);
    HIPCHK(launch_ttm_first_blocked(P.m[n].pelem, b.xb[n], b.xs[n], A, I, B, P.dims[P.N - 1], b.Ut64[n],
                                    P.m[n].R, b.u16, out, st));
  } else if (P.need_pad) {
    // precision form: the product reads the padded bf16 copy on bf16 MFMA
    HIPCHK(convert_tensor(E_F64, b.Ut64[n], E_BF16, b.Uop, P.m[n].R * I, st));
    ProfScope ps("ttm", st);
    HIPCHK(launch_ttm_padded(b.xpad, A, I, B, P.dims[P.N - 1], b.Uop, P.m[n].R, out, st));
  } else {
    HIPCHK(convert_tensor(E_F64, b.Ut64[n], P.telem, b.Uop, P.m[n].R * I, st));
    ProfScope ps("ttm", st);
    HIPCHK(launch_ttm(P.telem, xsrc, A, I, B, b.Uop, P.m[n].R, out, nullptr, 0, st));
  }
  return RBKI_OK;
}

// The explicit error of a Tucker model whose core (R_1 x ... x R_N, chain
// element type) is in chain buffer `which`: H = G x_2 U2 ... x_N UN through
// the chain buffers, then sum (x - U^(1) H)^2 and sum x^2 over X_(0) into
// sums (device, 2 doubles), copied to sums_host.
rbki_status reconstruct_error(const Plan& P, const Buffers& b, const void* X, int which, double* sums,
                              double* sums_host, hipStream_t st) {
  void* bufs[2] = {b.chainA, b.chainB};
  int64_t cur[8];
  for (int n = 0; n < P.N; ++n) cur[n] = P.ranks[n];
  void* src = bufs[which];
  int wsrc = which;
  for (int n = 1; n < P.N; ++n) {
    // expanding mode n: Y[a, i, b] = sum_r U[i, r] G[a, r, b]; launch_ttm
    // contracts the middle index (here of length R) against the rows of an
    // "Ut" whose rows are the output index, so U itself (I x R) is passed
    int64_t A = 1, B = 1;
    for (int k = 0; k < n; ++k) A *= cur[k];
    for (int k = n + 1; k < P.N; ++k) B *= cur[k];
    const int64_t R = P.m[n].R, I = P.m[n].I;
    HIPCHK(store_factor(b.Ut64[n], R, I, b.Uop, P.celem == E_F64 ? E_F64 : E_F32, st));
    void* dst = bufs[wsrc ^ 1];
    HIPCHK(launch_ttm(P.celem, src, A, R, B, b.Uop, I, dst, nullptr, 0, st));
    src = dst;
    wsrc ^= 1;
    cur[n] = I;
  }
  // residual over X_(0) with U^(1)
  {
    const int64_t I0 = P.dims[0], J0 = P.T / P.dims[0], R0 = P.m[0].R;
    HIPCHK(convert_tensor(E_F64, b.Ut64[0], P.celem, b.Uop, R0 * I0, st));
    ProfScope ps("error", st);
    // precision forms: U H from split bfloat16 operands, x and the sums exact
    HIPCHK(launch_residual(P.xelem, X, P.celem, b.Uop, src, I0, J0, R0, sums, b.rpartial, 0, st, P.need_pad));
  }
  HIPCHK(hipMemcpyAsync(sums_host, sums, 16, hipMemcpyDeviceToHost, st));
  return RBKI_OK;
}

// Alg. 2, step 6, a later product of the core chain: G <- G x_n U^(n)T from
// chain buffer `which` into the other one; cur holds G's dimensions.
rbki_status chain_product(const Plan& P, const Buffers& b, int n, int64_t* cur, int& which, hipStream_t st) {
  int64_t A = 1, B = 1;
  for (int k = 0; k < n; ++k) A *= cur[k];
  for (int k = n + 1; k < P.N; ++k) B *= cur[k];
  const int64_t I = cur[n];
  void* bufs[2] = {b.chainA, b.chainB};
  HIPCHK(convert_tensor(E_F64, b.Ut64[n], P.celem, b.Uop, P.m[n].R * I, st));
  HIPCHK(launch_ttm(P.celem, bufs[which], A, I, B, b.Uop, P.m[n].R, bufs[which ^ 1], nullptr, 0, st));
  which ^= 1;
  cur[n] = P.m[n].R;
  return RBKI_OK;
}

// The core chain runs the first mode, then the others in increasing order;
// the mode of its second product (-1 for one mode).
int second_chain_mode(const Plan& P) { return P.N < 2 ? -1 : (P.first_mode == 0 ? 1 : 0); }

// The second product of the core chain, on G_1 in chain buffer A (into B).
rbki_status second_product(const Plan& P, const Buffers& b, hipStream_t st) {
  int64_t cur[8];
  for (int n = 0; n < P.N; ++n) cur[n] = P.dims[n];
  cur[P.first_mode] = P.m[P.first_mode].R;
  int which = 0;
  return chain_product(P, b, second_chain_mode(P), cur, which, st);
}

// done: the number of the core chain's products already enqueued (0, 1 or 2,
// on streams that st has joined).
rbki_status run_core_and_error(const Plan& P, const Buffers& b, const void* X, const void* xsrc, void* core,
                               int out_elem, bool want_err, double* sums_host, void** core_out, hipStream_t st,
                               int done = 0) {
  int64_t cur[8];
  for (int n = 0; n < P.N; ++n) cur[n] = P.dims[n];
  void* bufs[2] = {b.chainA, b.chainB};
  int which = 0;
  // first product reads X
  if (done < 1) {
    rbki_status s = first_product(P, b, xsrc, st);
    if (s != RBKI_OK) return s;
  }
  cur[P.first_mode] = P.m[P.first_mode].R;
  int k = 1;                                       // products so far
  for (int n = 0; n < P.N; ++n) {
    if (n == P.first_mode) continue;
    if (k++ < done) {                              // enqueued beside the modes' work
      which ^= 1;
      cur[n] = P.m[n].R;
      continue;
    }
    rbki_status s = chain_product(P, b, n, cur, which, st);
    if (s != RBKI_OK) return s;
  }
  void* G = bufs[which];
  int64_t nc = 1;
  for (int n = 0; n < P.N; ++n) nc *= P.ranks[n];
  if (core) HIPCHK(convert_tensor(P.celem, G, out_elem, core, nc, st));
  if (core_out) {
    // the reconstruction chain below reuses both chain buffers
    HIPCHK(convert_tensor(P.celem, G, P.celem, b.gkeep, nc, st));
    *core_out = b.gkeep;
  }
  if (!want_err) return RBKI_OK;
  return reconstruct_error(P, b, X, which, b.sums, sums_host, st);
}

}  // namespace

// ====================================================================== ABI

size_t tucker_bytes(const rbki_params* prm, int xtype, const Plan& P);

extern "C" {

const char* rbki_version(void) { return "rbkitk 0.1 (gfx950)"; }

const char* rbki_last_error(void) { return g_err.c_str(); }

void rbki_profile_enable(int on) { g_prof_on = on != 0; }

void rbki_profile_reset(void) {
  prof_drain();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.clear();
}

rbki_status rbki_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
  if (!kernel) return fail(RBKI_E_INVALID, "kernel name is NULL");
  prof_drain();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  auto it = g_prof.find(kernel);
  if (launches) *launches = it == g_prof.end() ? 0 : it->second.launches;
  if (total_ms) *total_ms = it == g_prof.end() ? 0.0 : it->second.ms;
  return RBKI_OK;
}

rbki_status rbki_omega(uint64_t seed, int mode, int64_t J, int64_t S, int dtype, void* out, void* stream) {
  if (J < 0 || S < 0 || mode < 0) return fail(RBKI_E_INVALID, "negative size or mode");
  if (dtype != RBKI_F64 && dtype != RBKI_F32 && dtype != RBKI_BF16) return fail(RBKI_E_INVALID, "bad dtype");
  if (J * S > 0 && !out) return fail(RBKI_E_INVALID, "out is NULL");
  HIPCHK(launch_omega(dtype_elem(dtype), seed, mode, J * S, out, (hipStream_t)stream));
  return RBKI_OK;
}

rbki_status rbki_philox(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out, void* stream) {
  if (count < 0) return fail(RBKI_E_INVALID, "negative count");
  if (count > 0 && (!ctr || !out)) return fail(RBKI_E_INVALID, "NULL buffer");
  HIPCHK(launch_philox(ctr, count, seed, out, (hipStream_t)stream));
  return RBKI_OK;
}

size_t rbki_sym_eig_workspace(int64_t n) {
  if (n < 1 || n > 1200) return 0;
  return jacobi_work_bytes(n) + 512;
}

rbki_status rbki_sym_eig(const double* Z, int64_t n, double* lam, double* Vt, void* workspace, size_t ws_bytes,
                         int* sweeps, void* stream) {
  if (n < 1 || n > 1200) return fail(RBKI_E_INVALID, "n = %lld outside [1, 1200]", (long long)n);
  if (!Z || !lam || !Vt) return fail(RBKI_E_INVALID, "NULL matrix or output");
  const size_t need = rbki_sym_eig_workspace(n);
  if (!workspace || ws_bytes < need) return fail(RBKI_E_INVALID, "workspace %zu bytes < required %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  int* info = (int*)((char*)workspace + ((jacobi_work_bytes(n) + 255) & ~(size_t)255));
  {
    ProfScope ps("jacobi", st);
    HIPCHK(jacobi_eig(Z, n, lam, Vt, workspace, info, 40, st));
  }
  HIPCHK(canonical_sign_rows(Vt, n, n, st));
  if (getenv("RBKI_JACOBI_PROF")) {
    unsigned long long pr[6];
    HIPCHK(hipMemcpyAsync(pr, (char*)workspace + jacobi_work_bytes(n) - 256 + 3 * 8 * 8, sizeof(pr),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    fprintf(stderr, "[jacobi n=%lld] rounds %llu  us/round: stage %.2f gram %.2f inner %.2f apply %.2f gridsync %.2f\n",
            (long long)n, pr[5], pr[0] / 100.0 / pr[5], pr[1] / 100.0 / pr[5], pr[2] / 100.0 / pr[5],
            pr[3] / 100.0 / pr[5], pr[4] / 100.0 / pr[5]);
  }
  if (sweeps) {
    int h[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(h, info, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *sweeps = h[1];
    if (h[0]) return fail(RBKI_E_NOCONV, "Jacobi reached its sweep limit (%d sweeps)", h[1]);
  }
  return RBKI_OK;
}

size_t rbki_sym_eig_top_workspace(int64_t n, int64_t k) {
  if (!eig_top_ok(n, k)) return 0;
  return ((eig_top_work_bytes(n, k) + 255) & ~(size_t)255) + 256;   // + the solver's status
}

rbki_status rbki_sym_eig_top(const double* Z, int64_t n, int64_t k, double* lam, double* Vt, void* workspace,
                             size_t ws_bytes, void* stream) {
  if (!eig_top_ok(n, k))
    return fail(RBKI_E_INVALID, "need 1 <= k <= n <= 512 (n = %lld, k = %lld)", (long long)n, (long long)k);
  if (!Z || !lam || !Vt) return fail(RBKI_E_INVALID, "NULL matrix or output");
  const size_t need = rbki_sym_eig_top_workspace(n, k);
  if (!workspace || ws_bytes < need) return fail(RBKI_E_INVALID, "workspace %zu bytes < required %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  void* ws[1] = {workspace};
  int* info = (int*)((char*)workspace + ((eig_top_work_bytes(n, k) + 255) & ~(size_t)255));
  HIPCHK(fill_zero(info, 8, st));
  {
    ProfScope ps("eig", st);
    HIPCHK(eig_top_batched(1, &Z, &n, &k, &lam, &Vt, ws, &info, st));
  }
  HIPCHK(canonical_sign_rows(Vt, k, n, st));
  int h[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(h, info, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h[0]) return fail(RBKI_E_NOCONV, "the workgroups of the reduction did not meet within the spin limit");
  return RBKI_OK;
}

size_t rbki_basis_workspace(const rbki_params* prm, int xtype, int mode) {
  Plan P;
  if (make_plan(prm, xtype, P) != RBKI_OK) return 0;
  (void)mode;
  return plan_bytes(P);
}

rbki_status rbki_basis(const void* X, int xtype, const rbki_params* prm, int mode, double* Qt, int64_t* width,
                       void* workspace, size_t ws_bytes, void* stream) {
  Plan P;
  rbki_status s = make_plan(prm, xtype, P);
  if (s != RBKI_OK) return s;
  if (mode < 0 || mode >= P.N) return fail(RBKI_E_INVALID, "mode %d outside [0, %d)", mode, P.N);
  if (!X || !Qt) return fail(RBKI_E_INVALID, "NULL tensor or output");
  const size_t need = plan_bytes(P);
  if (!workspace || ws_bytes < need)
    return fail(RBKI_E_INVALID, "workspace %zu bytes < required %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  Arena ar(workspace, ws_bytes);
  Buffers b;
  carve(P, ar, b);
  dgemm_set_scratch(b.ln[0].dscratch, kDgemmScratch);
  const void* xsrc = X;
  if (P.need_pad) {
    ProfScope ps("convert", st);
    s = convert_input(P, b, X, st);
    if (s != RBKI_OK) return s;
  }
  HIPCHK(fill_zero(b.info, counters_bytes(P), st));
  s = run_mode(P, b, 0, xsrc, mode, false, st);
  if (s != RBKI_OK) return s;
  const ModeGeom& g = P.m[mode];
  // compact the kept basis vectors (rows whose norm is nonzero) into Qt
  const int64_t Sout = std::min<int64_t>(g.Sp, g.I);
  HIPCHK(row_norms2(b.Qt[mode], g.Sp, g.I, b.lam[mode], st));
  std::vector<double> nrm(g.Sp);
  HIPCHK(hipMemcpyAsync(nrm.data(), b.lam[mode], g.Sp * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int64_t w = 0;
  for (int64_t k = 0; k < g.Sp && w < Sout; ++k) {
    if (nrm[k] > 0.0) {
      HIPCHK(hipMemcpyAsync(Qt + w * g.I, b.Qt[mode] + k * g.I, g.I * 8, hipMemcpyDeviceToDevice, st));
      ++w;
    }
  }
  if (w < Sout) HIPCHK(fill_zero(Qt + w * g.I, (size_t)(Sout - w) * g.I * 8, st));
  HIPCHK(hipStreamSynchronize(st));
  if (width) *width = w;
  return RBKI_OK;
}

int64_t rbki_basis_rows(const rbki_params* prm, int xtype, int mode) {
  Plan P;
  if (make_plan(prm, xtype, P) != RBKI_OK || mode < 0 || mode >= P.N) return 0;
  return std::min<int64_t>(P.m[mode].Sp, P.m[mode].I);
}

size_t rbki_tucker_workspace(const rbki_params* prm, int xtype) {
  Plan P;
  if (make_plan(prm, xtype, P) != RBKI_OK) return 0;
  return tucker_bytes(prm, xtype, P);
}

}  // extern "C"

namespace rbki {
rbki_status finish_result(const HostResult& hr, double* rel_err) {
  if (rel_err) *rel_err = hr.sums[1] > 0 ? std::sqrt(hr.sums[0] / hr.sums[1]) : 0.0;
  for (int n = 0; n < hr.nmodes; ++n) {
    if (g_prof_on) {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof["jacobi_sweeps"].launches += hr.info[2 * n + 1];
    }
    if (hr.info[2 * n]) return fail(RBKI_E_NOCONV, "the eigen-solver did not finish in mode %d", n);
  }
  return RBKI_OK;
}

void set_error(rbki_status s, const char* msg) { fail(s, "%s", msg); }
}  // namespace rbki

// Helper streams of the current device for modes that run beside the
// caller's stream (created once, default priority, non-blocking).
static std::mutex g_lane_mu;
static std::map<int, std::vector<hipStream_t>> g_lane_pool;

static hipStream_t lane_stream(int lane) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_lane_mu);
  std::vector<hipStream_t>& v = g_lane_pool[dev];
  while ((int)v.size() < kMaxLanes - 1) {
    hipStream_t h = nullptr;
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) return nullptr;
    v.push_back(h);
  }
  return v[lane - 1];
}

// Alg. 2, steps 1-3 for every mode.  Mode n uses scratch set n % lanes; with
// more than one set the sets run on their own streams, forked from and
// joined back to st by events (the request server keeps one stream per
// request).  Each mode does the same work either way.
// inline_factors: each mode's factor step (and, for the first mode of the
// core chain, the first product) follows its Krylov chain on its stream, so
// that it runs beside the later modes' work; the chain's second product
// follows as soon as both its inputs are enqueued, on the stream of the later
// one after an event of the other.  *chain_done receives the number of the
// core chain's products enqueued.
static rbki_status run_modes(const Plan& P, const Buffers& b, const void* xsrc, hipStream_t st,
                             bool inline_factors = false, int* chain_done = nullptr) {
  if (chain_done) *chain_done = 0;
  if (P.fused) {
    // the sketch and Gram passes one after the other, each into its mode's
    // set, then every mode's Krylov chain in one launch
    ChainJob jobs[8];
    for (int n = 0; n < P.N; ++n) {
      rbki_status s = run_mode_heavy(P, b, n, xsrc, n, st);
      if (s != RBKI_OK) return s;
      jobs[n] = chain_job(P, b, n, n, (int)P.m[n].Sp);
    }
    return run_chains(P, jobs, P.N, 0, P.q, st);
  }
  const int lanes = (P.concurrent || P.one_stream) ? 1 : b.lanes;
  hipStream_t ls[kMaxLanes] = {st, st, st};
  hipEvent_t ev[kMaxLanes] = {};
  for (int l = 1; l < lanes; ++l) {
    ls[l] = lane_stream(l);
    if (!ls[l]) return fail(RBKI_E_HIP, "cannot create a helper stream");
  }
  if (lanes > 1) {
    for (int l = 0; l < lanes; ++l) HIPCHK(hipEventCreateWithFlags(&ev[l], hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev[0], st));
    for (int l = 1; l < lanes; ++l) HIPCHK(hipStreamWaitEvent(ls[l], ev[0], 0));
  }
  // the sketch and Gram kernels of successive modes one after the other,
  // the Krylov steps beside them
  hipEvent_t heavy[8] = {};
  if (lanes > 1)
    for (int n = 0; n < P.N; ++n) HIPCHK(hipEventCreateWithFlags(&heavy[n], hipEventDisableTiming));
  // the second product of the core chain: its factor's mode and the first
  // product, each with an event for the other's stream
  const int n2 = inline_factors && lanes > 1 ? second_chain_mode(P) : -1;
  hipEvent_t ev_first = nullptr, ev_fac2 = nullptr;
  bool first_enq = false, fac2_enq = false;
  int products = 0;
  if (n2 >= 0) {
    HIPCHK(hipEventCreateWithFlags(&ev_first, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_fac2, hipEventDisableTiming));
  }
  // With several scratch sets, the modes of a round (one per set) are enqueued
  // heavy phases first, so that the next mode's sketch and Gram kernels are
  // queued before the long chain of small Krylov kernels of the previous one.
  // A mode's chain follows its own heavy phase on its stream; modes sharing a
  // set keep their order.
  rbki_status s = RBKI_OK;
  if (lanes == 1) {
    for (int n = 0; n < P.N && s == RBKI_OK; ++n) s = run_mode(P, b, n % b.lanes, xsrc, n, true, st);
  } else {
    for (int n0 = 0; n0 < P.N && s == RBKI_OK; n0 += lanes) {
      const int n1 = std::min(P.N, n0 + lanes);
      for (int n = n0; n < n1 && s == RBKI_OK; ++n)
        s = run_mode_heavy(P, b, n % lanes, xsrc, n, ls[n % lanes], n > 0 ? heavy[n - 1] : nullptr, heavy[n]);
      for (int n = n0; n < n1 && s == RBKI_OK; ++n) {
        hipStream_t ln = ls[n % lanes];
        s = run_mode_chain(P, b, n % lanes, n, true, ln);
        if (s == RBKI_OK && inline_factors) s = factor_one(P, b, n, ln);
        if (s == RBKI_OK && inline_factors && n == P.first_mode) {
          s = first_product(P, b, xsrc, ln);
          products = 1;
          first_enq = true;
          if (s == RBKI_OK && n2 >= 0) HIPCHK(hipEventRecord(ev_first, ln));
        }
        if (s == RBKI_OK && n == n2) {
          fac2_enq = true;
          HIPCHK(hipEventRecord(ev_fac2, ln));
        }
        if (s == RBKI_OK && n2 >= 0 && products == 1 && first_enq && fac2_enq) {
          // this stream has just enqueued the later of the two inputs
          HIPCHK(hipStreamWaitEvent(ln, n == n2 ? ev_first : ev_fac2, 0));
          s = second_product(P, b, ln);
          products = 2;
        }
      }
    }
  }
  if (lanes > 1) {
    for (int l = 1; l < lanes; ++l) {
      HIPCHK(hipEventRecord(ev[l], ls[l]));
      HIPCHK(hipStreamWaitEvent(st, ev[l], 0));
    }
    for (int l = 0; l < lanes; ++l) HIPCHK(hipEventDestroy(ev[l]));
    for (int n = 0; n < P.N; ++n) HIPCHK(hipEventDestroy(heavy[n]));
    if (ev_first) HIPCHK(hipEventDestroy(ev_first));
    if (ev_fac2) HIPCHK(hipEventDestroy(ev_fac2));
  }
  if (chain_done && inline_factors) *chain_done = products;
  dgemm_set_scratch(b.ln[0].dscratch, kDgemmScratch);
  return s;
}

// ------------------------------------------------------------ sequential truncation
// Stage n of the sequential form runs mode n of Y_{n-1} (Y_0 = X) with the
// same kernels as an independent-mode solve of that tensor, then forms
// Y_n = Y_{n-1} x_n U^(n)T.  Workspace: the factors, the core, the error sums
// and the stage status kept for the whole solve; two buffers for the
// successive Y; one region reused by every stage's scratch (and, at the end,
// by the reconstruction of the error).
struct SeqLayout {
  Plan st[8];
  int64_t sdims[8][8];       // dims of each stage's tensor
  rbki_params sp[8];         // each stage's problem statement
  int yelem = E_F32;         // element type of the intermediates
  size_t fac[8] = {}, gkeep = 0, sums = 0, info = 0, ya = 0, yb = 0, stage = 0, stage_bytes = 0, total = 0;
};

rbki_status seq_layout(const rbki_params* prm, int xtype, const Plan& P0, SeqLayout& L) {
  L.yelem = P0.xelem == E_F64 ? E_F64 : E_F32;
  const int yt = L.yelem == E_F64 ? RBKI_F64 : RBKI_F32;
  int64_t cur[8];
  for (int n = 0; n < P0.N; ++n) cur[n] = P0.dims[n];
  int64_t ymax = 1;
  for (int n = 0; n < P0.N; ++n) {
    for (int k = 0; k < P0.N; ++k) L.sdims[n][k] = cur[k];
    L.sp[n] = *prm;
    L.sp[n].dims = L.sdims[n];
    L.sp[n].truncation = RBKI_INDEPENDENT;
    if (n > 0) L.sp[n].precision = RBKI_PLAIN;
    rbki_status s = make_plan(&L.sp[n], n == 0 ? xtype : yt, L.st[n]);
    if (s != RBKI_OK) return s;
    L.st[n].concurrent = P0.concurrent;
    L.stage_bytes = std::max(L.stage_bytes, plan_bytes(L.st[n]));
    cur[n] = P0.ranks[n];
    int64_t t = 1;
    for (int k = 0; k < P0.N; ++k) t *= cur[k];
    ymax = std::max(ymax, t);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) { off = (off + 255) & ~(size_t)255; size_t o = off; off += bytes; return o; };
  for (int n = 0; n < P0.N; ++n) L.fac[n] = take((size_t)P0.m[n].R * P0.m[n].I * 8);
  int64_t nc = 1;
  for (int n = 0; n < P0.N; ++n) nc *= P0.ranks[n];
  L.gkeep = take((size_t)nc * 8);
  L.sums = take(64);
  L.info = take(256);
  L.ya = take((size_t)ymax * elem_size(L.yelem));
  L.yb = take((size_t)ymax * elem_size(L.yelem));
  L.stage = take(L.stage_bytes);
  L.total = off + 256;
  return RBKI_OK;
}

// The whole sequential solve on `st`.  On return b holds the factors (Ut64)
// and the error sums, *core_chain the core in the chain element type of P0
// (for Alg. 3), hr the sums and the solver status (copied when st reaches
// them).
rbki_status sequential_enqueue(const void* X, const rbki_params* prm, int xtype, const Plan& P0, void* core,
                               void* const* factors, int out_type, char* ws, bool want_err, Buffers& b,
                               void** core_chain, HostResult* hr, hipStream_t st) {
  SeqLayout L;
  rbki_status s = seq_layout(prm, xtype, P0, L);
  if (s != RBKI_OK) return s;
  double* fac[8];
  for (int n = 0; n < P0.N; ++n) fac[n] = (double*)(ws + L.fac[n]);
  int* info = (int*)(ws + L.info);
  HIPCHK(fill_zero(info, 256, st));
  void* ybuf[2] = {ws + L.ya, ws + L.yb};
  const void* src = X;
  int src_elem = P0.xelem;
  for (int n = 0; n < P0.N; ++n) {
    const Plan& Pn = L.st[n];
    Arena ar(ws + L.stage, L.stage_bytes);
    Buffers bn;
    carve(Pn, ar, bn);
    dgemm_set_scratch(bn.ln[0].dscratch, kDgemmScratch);
    if (Pn.need_pad) {
      ProfScope ps("convert", st);
      s = convert_input(Pn, bn, src, st);
      if (s != RBKI_OK) return s;
    }
    HIPCHK(fill_zero(bn.info, counters_bytes(Pn), st));
    s = run_mode(Pn, bn, 0, src, n, true, st);
    if (s != RBKI_OK) return s;
    s = factor_single(Pn, bn, n, st);
    if (s != RBKI_OK) return s;
    const ModeGeom& g = Pn.m[n];
    HIPCHK(copy_rows_f64(fac[n], g.I, bn.Ut64[n], g.I, g.R, g.I, st));
    HIPCHK(hipMemcpyAsync(info + 2 * n, bn.info + 2 * n, 2 * sizeof(int), hipMemcpyDeviceToDevice, st));
    // Y_n = Y_{n-1} x_n U^(n)T, in float32 (float64 for a float64 X)
    HIPCHK(convert_tensor(E_F64, fac[n], src_elem, bn.Uop, g.R * g.I, st));
    void* dst = ybuf[n & 1];
    {
      ProfScope ps("ttm", st);
      HIPCHK(launch_ttm(src_elem, src, g.A, g.I, g.B, bn.Uop, g.R, dst, nullptr, 0, st));
    }
    src = dst;
    src_elem = L.yelem;
  }
  // the core is Y_N; its copy in the chain element type for Alg. 3
  int64_t nc = 1;
  for (int n = 0; n < P0.N; ++n) nc *= P0.ranks[n];
  if (core) HIPCHK(convert_tensor(L.yelem, src, dtype_elem(out_type), core, nc, st));
  for (int n = 0; n < P0.N; ++n)
    if (factors && factors[n])
      HIPCHK(store_factor(fac[n], P0.m[n].R, P0.m[n].I, factors[n], dtype_elem(out_type), st));
  void* gk = ws + L.gkeep;
  HIPCHK(convert_tensor(L.yelem, src, P0.celem, gk, nc, st));
  if (core_chain) *core_chain = gk;
  // the error of the returned model, with the first stage's buffers
  Arena ar(ws + L.stage, L.stage_bytes);
  carve(P0, ar, b);
  for (int n = 0; n < P0.N; ++n) b.Ut64[n] = fac[n];
  b.sums = (double*)(ws + L.sums);
  b.info = info;
  if (want_err) {
    HIPCHK(convert_tensor(P0.celem, gk, P0.celem, b.chainA, nc, st));
    s = reconstruct_error(P0, b, X, 0, b.sums, hr->sums, st);
    if (s != RBKI_OK) return s;
  }
  HIPCHK(hipMemcpyAsync(hr->info, info, 2 * P0.N * sizeof(int), hipMemcpyDeviceToHost, st));
  hr->nmodes = P0.N;
  return RBKI_OK;
}

// Workspace of a decomposition: the independent form's plan, or the
// sequential form's layout.
size_t tucker_bytes(const rbki_params* prm, int xtype, const Plan& P) {
  if (!P.sequential) return plan_bytes(P);
  SeqLayout L;
  if (seq_layout(prm, xtype, P, L) != RBKI_OK) return 0;
  return L.total;
}

// ------------------------------------------------------------ adaptive q
// rBKI-TK with q chosen by the stopping rule of Sec. 4: after every Krylov
// step t (all modes), the rank-k approximation and its Fit to X; stop once
// two consecutive Fits differ by at most fit_tol.  Each mode's Gram matrix
// (and a sampled mode's Y Y^T) and the products C Q of its basis blocks are
// kept across the steps, so X is read by the sketch / Gram pass once, and by
// the core and the error once per step.
struct AdaptiveLayout {
  size_t C[8] = {}, CY[8] = {}, CQ[8] = {};
  size_t total = 0;
};

int adaptive_q(const rbki_params* prm, const Plan& P) {
  // beyond ceil(I_n / S_n) steps every basis spans its mode space, and the
  // Fit stops changing: the rule stops there at the latest
  int64_t qmax = 0;
  for (int n = 0; n < P.N; ++n) qmax = std::max<int64_t>(qmax, ceil_div(P.m[n].I, P.m[n].S));
  int64_t q = std::min<int64_t>(prm->power, qmax);
  for (int n = 0; n < P.N; ++n) q = std::min<int64_t>(q, 1200 / P.m[n].S - 1);
  return (int)std::max<int64_t>(q, 0);
}

rbki_status adaptive_plan(const rbki_params* prm, int xtype, Plan& P, rbki_params& pa, AdaptiveLayout& L) {
  Plan P0;
  rbki_status s = make_plan(prm, xtype, P0);
  if (s != RBKI_OK) return s;
  if (P0.power || P0.sequential)
    return fail(RBKI_E_UNSUPPORTED, "the stopping rule is built for the Krylov variant with independent modes");
  pa = *prm;
  pa.power = adaptive_q(prm, P0);
  s = make_plan(&pa, xtype, P);
  if (s != RBKI_OK) return s;
  size_t off = plan_bytes(P);
  auto take = [&](size_t bytes) { off = (off + 255) & ~(size_t)255; size_t o = off; off += bytes; return o; };
  for (int n = 0; n < P.N; ++n) {
    const ModeGeom& g = P.m[n];
    L.C[n] = take((size_t)g.I * g.I * 8);
    if (g.sampled) L.CY[n] = take((size_t)g.I * g.I * 8);
    L.CQ[n] = take((size_t)g.Sp * g.I * 8);
  }
  L.total = off + 256;
  return RBKI_OK;
}

rbki_status adaptive_impl(const void* X, int xtype, const rbki_params* prm, double fit_tol, void* core,
                          void* const* factors, int out_type, void* workspace, size_t ws_bytes, double* rel_err,
                          int* q_used, hipStream_t st) {
  Plan P;
  rbki_params pa;
  AdaptiveLayout AL;
  rbki_status s = adaptive_plan(prm, xtype, P, pa, AL);
  if (s != RBKI_OK) return s;
  if (!X) return fail(RBKI_E_INVALID, "X is NULL");
  if (out_type != RBKI_F64 && out_type != RBKI_F32) return fail(RBKI_E_INVALID, "out_type must be F64 or F32");
  if (!(fit_tol == fit_tol)) return fail(RBKI_E_INVALID, "fit_tol is NaN");
  if (!workspace || ws_bytes < AL.total)
    return fail(RBKI_E_INVALID, "workspace %zu bytes < required %zu", ws_bytes, AL.total);
  char* ws = (char*)workspace;
  Arena ar(workspace, ws_bytes);
  Buffers b;
  carve(P, ar, b);
  const Lane& L0 = b.ln[0];
  if (P.need_pad) {
    ProfScope ps("convert", st);
    s = convert_input(P, b, X, st);
    if (s != RBKI_OK) return s;
  }
  HIPCHK(fill_zero(b.info, counters_bytes(P), st));
  double *Cm[8], *CYm[8], *CQm[8];
  for (int n = 0; n < P.N; ++n) {
    const ModeGeom& g = P.m[n];
    Cm[n] = (double*)(ws + AL.C[n]);
    CYm[n] = g.sampled ? (double*)(ws + AL.CY[n]) : nullptr;
    CQm[n] = (double*)(ws + AL.CQ[n]);
    if (P.fused) {
      // each mode's Gram pass into its own chain set, which keeps C and the
      // products C Q for every step
      s = run_mode_heavy(P, b, n, X, n, st);
      if (s != RBKI_OK) return s;
      continue;
    }
    // the Gram pass (and the sample's), kept for every step; block 0
    s = run_mode_heavy(P, b, 0, X, n, st);
    if (s != RBKI_OK) return s;
    HIPCHK(copy_rows_f64(Cm[n], g.I, L0.C, g.I, g.I, g.I, st));
    if (g.sampled) HIPCHK(copy_rows_f64(CYm[n], g.I, L0.CY, g.I, g.I, g.I, st));
    s = krylov_block0(P, b, L0, n, st);
    if (s != RBKI_OK) return s;
  }
  dgemm_set_scratch(L0.dscratch, kDgemmScratch);
  HostResult hr;
  double fit_prev = 0.0, err = 0.0;
  int t = 0;
  for (;; ++t) {
    if (P.fused) {
      // block t of every mode's basis and Z over the t + 1 blocks, in one
      // launch: the same steps as the fixed-q launch, one block at a time
      ChainJob jobs[8];
      for (int n = 0; n < P.N; ++n) jobs[n] = chain_job(P, b, n, n, (int)(P.m[n].S * (t + 1)));
      s = run_chains(P, jobs, P.N, t, t, st);
      if (s != RBKI_OK) return s;
    }
    for (int n = 0; n < P.N; ++n) {
      const ModeGeom& g = P.m[n];
      const int64_t I = g.I, S = g.S, m = S * (t + 1);
      if (P.fused) {
        s = factor_single(P, b, n, st, m);
        if (s != RBKI_OK) return s;
        continue;
      }
      if (t > 0) {
        // Krylov step t (Alg. 1); a mode that is not sampled takes C Q_{t-1}
        // from the products kept for Z
        s = krylov_step(P, b, L0, n, t, g.sampled ? CYm[n] : Cm[n], g.sampled ? nullptr : CQm[n], !g.sampled, st);
        if (s != RBKI_OK) return s;
      }
      // C Q_t, then Z_t = Q^T C Q over the t + 1 blocks (Alg. 2, step 3)
      HIPCHK(dgemm(0, 0, S, I, I, 1.0, b.Qt[n] + (m - S) * I, I, Cm[n], I, 0.0, CQm[n] + (m - S) * I, I, st));
      HIPCHK(dgemm(0, 1, m, m, I, 1.0, b.Qt[n], I, CQm[n], I, 0.0, b.Z[n], m, st));
      s = factor_single(P, b, n, st, m);
      if (s != RBKI_OK) return s;
    }
    void* gk = nullptr;
    s = run_core_and_error(P, b, X, X, nullptr, dtype_elem(out_type), true, hr.sums, &gk, st);
    if (s != RBKI_OK) return s;
    HIPCHK(hipMemcpyAsync(hr.info, b.info, 2 * P.N * sizeof(int), hipMemcpyDeviceToHost, st));
    hr.nmodes = P.N;
    HIPCHK(hipStreamSynchronize(st));
    s = finish_result(hr, &err);
    if (s != RBKI_OK) return s;
    const double fit = 1.0 - err;     // Fit of Sec. 4, as a fraction, against X
    if ((t > 0 && fabs(fit - fit_prev) <= fit_tol) || t >= P.q) break;
    fit_prev = fit;
  }
  int64_t nc = 1;
  for (int n = 0; n < P.N; ++n) nc *= P.ranks[n];
  if (core) HIPCHK(convert_tensor(P.celem, b.gkeep, dtype_elem(out_type), core, nc, st));
  for (int n = 0; n < P.N; ++n)
    if (factors && factors[n])
      HIPCHK(store_factor(b.Ut64[n], P.m[n].R, P.m[n].I, factors[n], dtype_elem(out_type), st));
  HIPCHK(hipStreamSynchronize(st));
  if (rel_err) *rel_err = err;
  if (q_used) *q_used = t;
  return RBKI_OK;
}

static rbki_status tucker_impl(const void* X, int xtype, const rbki_params* prm, void* core, void* const* factors,
                        int out_type, void* workspace, size_t ws_bytes, double* rel_err, hipStream_t st, Plan& P,
                        Buffers& b, void** core_chain, HostResult* async_res, bool one_stream = false,
                        bool served = false) {
  rbki_status s = make_plan(prm, xtype, P);
  if (s != RBKI_OK) return s;
  P.concurrent = served;                       // enqueued by the request server
  P.one_stream = one_stream;
  if (!X) return fail(RBKI_E_INVALID, "X is NULL");
  if (out_type != RBKI_F64 && out_type != RBKI_F32) return fail(RBKI_E_INVALID, "out_type must be F64 or F32");
  const size_t need = tucker_bytes(prm, xtype, P);
  if (need == 0) return fail(RBKI_E_INVALID, "%s", g_err.c_str());
  if (!workspace || ws_bytes < need)
    return fail(RBKI_E_INVALID, "workspace %zu bytes < required %zu", ws_bytes, need);
  if (P.sequential) {
    HostResult local;
    HostResult* hr = async_res ? async_res : &local;
    s = sequential_enqueue(X, prm, xtype, P, core, factors, out_type, (char*)workspace, rel_err || async_res, b,
                           core_chain, hr, st);
    if (s != RBKI_OK || async_res) return s;
    HIPCHK(hipStreamSynchronize(st));
    return finish_result(*hr, rel_err);
  }
  Arena ar(workspace, ws_bytes);
  carve(P, ar, b);
  dgemm_set_scratch(b.ln[0].dscratch, kDgemmScratch);
  const void* xsrc = X;
  if (P.need_pad) {
    ProfScope ps("convert", st);
    s = convert_input(P, b, X, st);
    if (s != RBKI_OK) return s;
  }
  HIPCHK(fill_zero(b.info, counters_bytes(P), st));
  // with concurrent modes, each mode's eigenproblem and factor (and the first
  // product of the core chain) run on its stream as soon as its Krylov basis
  // is done
  bool inline_factors = !P.concurrent && !P.one_stream && !P.fused && b.lanes > 1;
  for (int n = 0; n < P.N; ++n) inline_factors = inline_factors && eig_top_ok(P.m[n].Sp, P.m[n].R);
  int chain_done = 0;
  s = run_modes(P, b, xsrc, st, inline_factors, &chain_done);
  if (s != RBKI_OK) return s;
  if (!inline_factors) {
    s = run_factors(P, b, st);
    if (s != RBKI_OK) return s;
  }
  for (int n = 0; n < P.N; ++n)
    if (factors && factors[n])
      HIPCHK(store_factor(b.Ut64[n], P.m[n].R, P.m[n].I, factors[n], dtype_elem(out_type), st));
  HostResult local;
  HostResult* hr = async_res ? async_res : &local;
  const bool want_err = rel_err || async_res;
  s = run_core_and_error(P, b, X, xsrc, core, dtype_elem(out_type), want_err, hr->sums, core_chain, st,
                         chain_done);
  if (s != RBKI_OK) return s;
  // the eigen-solver's status comes back whether or not the error was asked
  // for, so a failed solve is never returned as RBKI_OK
  HIPCHK(hipMemcpyAsync(hr->info, b.info, 2 * P.N * sizeof(int), hipMemcpyDeviceToHost, st));
  hr->nmodes = P.N;
  if (async_res) return RBKI_OK;              // the caller reads the results after the stream completes
  HIPCHK(hipStreamSynchronize(st));
  return finish_result(*hr, want_err ? rel_err : nullptr);
}


namespace rbki {
rbki_status tucker_enqueue(const void* X, int xtype, const rbki_params* prm, void* core, void* const* factors,
                           int out_type, void* workspace, size_t ws_bytes, hipStream_t st, HostResult* hr) {
  Plan P;
  Buffers b;
  return tucker_impl(X, xtype, prm, core, factors, out_type, workspace, ws_bytes, nullptr, st, P, b, nullptr, hr,
                     false, true);
}
}  // namespace rbki

extern "C" {

// Releases what the library holds between calls: the helper streams of the
// concurrent modes (after their work is done) and the events of pending
// timing records.  Makes no HIP call when it holds nothing.
void rbki_release(void) {
  prof_drain();
  std::lock_guard<std::mutex> lk(g_lane_mu);
  if (g_lane_pool.empty()) return;
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : g_lane_pool) {
    if (hipSetDevice(kv.first) != hipSuccess) continue;
    for (hipStream_t h : kv.second) {
      (void)hipStreamSynchronize(h);
      (void)hipStreamDestroy(h);
    }
  }
  if (have_cur) (void)hipSetDevice(cur);
  g_lane_pool.clear();
}

size_t rbki_tucker_result_bytes(void) { return sizeof(rbki::HostResult); }

rbki_status rbki_tucker_enqueue(const void* X, int xtype, const rbki_params* prm, void* core, void* const* factors,
                                int out_type, void* workspace, size_t ws_bytes, void* result, void* stream) {
  if (!result) return fail(RBKI_E_INVALID, "result is required");
  rbki::HostResult* hr = (rbki::HostResult*)result;
  hr->nmodes = 0;
  Plan P;
  Buffers b;
  // the solo configuration (the modes on helper streams beside the caller's),
  // as rbki_tucker, without its final wait
  return tucker_impl(X, xtype, prm, core, factors, out_type, workspace, ws_bytes, nullptr, (hipStream_t)stream, P,
                     b, nullptr, hr);
}

rbki_status rbki_tucker_result(const void* result, double* rel_err) {
  if (!result) return fail(RBKI_E_INVALID, "result is required");
  return rbki::finish_result(*(const rbki::HostResult*)result, rel_err);
}

rbki_status rbki_tucker(const void* X, int xtype, const rbki_params* prm, void* core, void* const* factors,
                        int out_type, void* workspace, size_t ws_bytes, double* rel_err, void* stream) {
  Plan P;
  Buffers b;
  return tucker_impl(X, xtype, prm, core, factors, out_type, workspace, ws_bytes, rel_err, (hipStream_t)stream, P,
                     b, nullptr, nullptr);
}

}  // extern "C"

// ------------------------------------------------------------ fixed device scratch
// For callers that cannot allocate: rbki_tucker with its workspace in this
// array.  Each device that loads the library holds its own copy for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static rbki_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(RBKI_E_UNSUPPORTED, "device %d: at most 64 devices", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RBKI_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RBKI_OK;
}

extern "C" {

size_t rbki_tucker_noalloc_limit(void) { return kScratchBytes; }

rbki_status rbki_tucker_noalloc(const void* X, int xtype, const rbki_params* prm, void* core, void* const* factors,
                                int out_type, double* rel_err, void* stream) {
  Plan P;
  rbki_status s = make_plan(prm, xtype, P);
  if (s != RBKI_OK) return s;
  const size_t need = tucker_bytes(prm, xtype, P);
  if (need == 0) return fail(RBKI_E_INVALID, "%s", g_err.c_str());
  if (need > kScratchBytes)
    return fail(RBKI_E_INVALID, "this problem needs %zu bytes of scratch; the fixed device scratch holds %zu", need,
                kScratchBytes);
  void* ws = nullptr;
  s = scratch_address(&ws);
  if (s != RBKI_OK) return s;
  Buffers b;
  return tucker_impl(X, xtype, prm, core, factors, out_type, ws, kScratchBytes, rel_err, (hipStream_t)stream, P, b,
                     nullptr, nullptr, true);
}

size_t rbki_tucker_adaptive_workspace(const rbki_params* prm, int xtype) {
  Plan P;
  rbki_params pa;
  AdaptiveLayout L;
  if (adaptive_plan(prm, xtype, P, pa, L) != RBKI_OK) return 0;
  return L.total;
}

rbki_status rbki_tucker_adaptive(const void* X, int xtype, const rbki_params* prm, double fit_tol, void* core,
                                 void* const* factors, int out_type, void* workspace, size_t ws_bytes,
                                 double* rel_err, int* q_used, void* stream) {
  return adaptive_impl(X, xtype, prm, fit_tol, core, factors, out_type, workspace, ws_bytes, rel_err, q_used,
                       (hipStream_t)stream);
}

// ---------------------------------------------------------------- Alg. 3
static bool htr_sizes(const Plan& P, const int64_t* tr, int64_t* r) {
  // r[0..N]: r[0] = r_N closing rank, r[k] = tr[k-1]
  r[0] = tr[P.N - 1];
  for (int k = 0; k < P.N; ++k) r[k + 1] = tr[k];
  for (int k = 0; k <= P.N; ++k)
    if (r[k] < 1) return false;
  return true;
}

static size_t htr_bytes(const rbki_params* prm, int xtype, const int64_t* tr_ranks, bool als) {
  Plan P;
  if (make_plan(prm, xtype, P) != RBKI_OK || !tr_ranks) return 0;
  int64_t r[9];
  if (!htr_sizes(P, tr_ranks, r)) return 0;
  int64_t S[8];
  for (int n = 0; n < P.N; ++n) S[n] = P.ranks[n];
  const size_t base = tucker_bytes(prm, xtype, P);
  if (base == 0) return 0;
  size_t extra = 0;
  for (int n = 0; n < P.N; ++n) extra += ((size_t)r[n] * S[n] * r[n + 1] * 8 + 255) & ~(size_t)255;
  extra += tr_svd_work_bytes(P.N, S, r) + tr_gap2_work_bytes(P.N, S, r) + 1024;
  if (als) extra += tr_als_work_bytes(P.N, S, r) + 256;
  return base + extra;
}

size_t rbki_htr_workspace(const rbki_params* prm, int xtype, const int64_t* tr_ranks) {
  return htr_bytes(prm, xtype, tr_ranks, false);
}

size_t rbki_htr_als_workspace(const rbki_params* prm, int xtype, const int64_t* tr_ranks) {
  return htr_bytes(prm, xtype, tr_ranks, true);
}

// Alg. 3: the Tucker step, then TR-SVD of the core (or, with als, TR-ALS
// sweeps from a start of the sketch stream), then X_n = G_n x_2 U^(n).
static rbki_status htr_impl(const void* X, int xtype, const rbki_params* prm, const int64_t* tr_ranks,
                            void* const* tr_cores, int out_type, void* workspace, size_t ws_bytes, double* rel_err,
                            bool als, int max_sweeps, double fit_tol, int* sweeps, hipStream_t st) {
  Plan P;
  rbki_status s = make_plan(prm, xtype, P);
  if (s != RBKI_OK) return s;
  if (!tr_ranks || !tr_cores) return fail(RBKI_E_INVALID, "NULL tr_ranks or tr_cores");
  int64_t r[9];
  if (!htr_sizes(P, tr_ranks, r)) return fail(RBKI_E_INVALID, "TR ranks must be >= 1");
  for (int k = 0; k <= P.N; ++k)
    if (r[k] > 64) return fail(RBKI_E_UNSUPPORTED, "TR rank %lld > 64", (long long)r[k]);
  for (int n = 0; n < P.N; ++n)
    if (!tr_cores[n]) return fail(RBKI_E_INVALID, "tr_cores[%d] is NULL", n);
  if (als && (max_sweeps < 0 || max_sweeps > 1000 || !(fit_tol == fit_tol)))
    return fail(RBKI_E_INVALID, "max_sweeps %d outside [0, 1000] or fit_tol NaN", max_sweeps);
  const size_t need = htr_bytes(prm, xtype, tr_ranks, als);
  if (!workspace || ws_bytes < need) return fail(RBKI_E_INVALID, "workspace %zu bytes < required %zu", ws_bytes, need);
  Buffers b;
  void* Gchain = nullptr;
  double e_tk = 0.0;
  s = tucker_impl(X, xtype, prm, nullptr, nullptr, RBKI_F64, workspace, ws_bytes, rel_err ? &e_tk : nullptr, st, P, b,
                  &Gchain, nullptr);
  if (s != RBKI_OK && s != RBKI_E_NOCONV) return s;
  // the remaining workspace after the Tucker plan
  size_t off = (tucker_bytes(prm, xtype, P) + 255) & ~(size_t)255;
  char* base = (char*)workspace + off;
  int64_t S[8];
  for (int n = 0; n < P.N; ++n) S[n] = P.ranks[n];
  double* cores[8];
  for (int n = 0; n < P.N; ++n) {
    cores[n] = (double*)base;
    base += ((size_t)r[n] * S[n] * r[n + 1] * 8 + 255) & ~(size_t)255;
  }
  const size_t tw = tr_svd_work_bytes(P.N, S, r);
  double* twork = (double*)base;
  base += (tw + 255) & ~(size_t)255;
  double* gwork = (double*)base;
  base += (tr_gap2_work_bytes(P.N, S, r) + 255) & ~(size_t)255;
  double* small = (double*)base;   // [0..1]: gap2, discarded; int info at +64
  base += 1024;
  HIPCHK(tr_svd_device(Gchain, P.celem, P.N, S, r, cores, twork, tw, (int*)(small + 8), small + 1, st));
  int sw = 0;
  if (als) {
    // TR-ALS from its own start (the sketch stream, tag 2); tr_svd_device
    // left the core in float64 at the start of its work area
    double err2 = 0.0;
    HIPCHK(tr_als_device(twork, P.N, S, r, cores, P.seed, max_sweeps, fit_tol, base, (int*)(small + 10), &sw, &err2,
                         st));
  }
  if (sweeps) *sweeps = sw;
  for (int n = 0; n < P.N; ++n)
    HIPCHK(tr_attach(cores[n], b.Ut64[n], r[n], S[n], r[n + 1], P.dims[n], tr_cores[n], dtype_elem(out_type), st));
  if (rel_err) {
    // ||X - TR||^2 = ||X - [[G;U]]||^2 + ||G - TR(G_n)||^2 (orthonormal U)
    HIPCHK(tr_gap2(Gchain, P.celem, P.N, S, r, cores, gwork, small, st));
    double gap2 = 0.0, sums[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&gap2, small, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sums, b.sums, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *rel_err = sums[1] > 0 ? std::sqrt((sums[0] + gap2) / sums[1]) : 0.0;
  }
  return s;
}

rbki_status rbki_htr(const void* X, int xtype, const rbki_params* prm, const int64_t* tr_ranks,
                     void* const* tr_cores, int out_type, void* workspace, size_t ws_bytes, double* rel_err,
                     void* stream) {
  return htr_impl(X, xtype, prm, tr_ranks, tr_cores, out_type, workspace, ws_bytes, rel_err, false, 0, 0.0, nullptr,
                  (hipStream_t)stream);
}

rbki_status rbki_htr_als(const void* X, int xtype, const rbki_params* prm, const int64_t* tr_ranks, int max_sweeps,
                         double fit_tol, void* const* tr_cores, int out_type, void* workspace, size_t ws_bytes,
                         double* rel_err, int* sweeps, void* stream) {
  return htr_impl(X, xtype, prm, tr_ranks, tr_cores, out_type, workspace, ws_bytes, rel_err, true, max_sweeps,
                  fit_tol, sweeps, (hipStream_t)stream);
}

}  // extern "C"
