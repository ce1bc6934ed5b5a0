// TR-SVD of the small Tucker core and the factor contraction of Alg. 3.
//
// TR-SVD (the method Alg. 3 cites for its "or using TR-SVD" branch), with fixed
// TR ranks (r_1 .. r_N) and closing rank r_0 = r_N:
//   1. unfold G as S_1 x (S_2 .. S_N); its leading r_0 r_1 left singular
//      vectors (zero beyond the rank) give core 1 as (r_0, S_1, r_1) with
//      column c = a0 r_1 + a1; the remainder U^T M is reshaped to
//      (r_0, r_1, S_2 .. S_N) and its r_0 axis moved last;
//   2. for k = 2 .. N-1 the remainder, unfolded as (r_{k-1} S_k) x rest,
//      gives core k from its leading r_k left singular vectors (reshaped to
//      (r_{k-1}, S_k, r_k)) and the next remainder U^T M;
//   3. the last remainder is core N, (r_{N-1}, S_N, r_0).
// Left singular vectors come from the eigenvectors of the Gram matrix M M^T,
// only the leading ones each step keeps (the leading-eigenpair solver:
// tridiagonal reduction, bisection, inverse iteration; one-sided Jacobi for
// Gram matrices beyond its sizes), all in float64, each signed so that its largest-
// magnitude entry is positive: with r_0 > 1 the first step files vector c
// under the pair (a0, a1), and a sign change there is not an orthogonal change
// of the next unfolding, so the sweep is only a function of G once signs are
// fixed.  The discarded energy is the trace of
// M M^T minus the kept eigenvalues, summed over the steps.
#include "rbki_kernels.h"

namespace rbki {

namespace {

inline unsigned gridn(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 8192)); }

template <class T>
__global__ void to_double_kernel(const T* src, double* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

// core1[a0, i, a1] = Vt[a0*r1 + a1][i] (rows of Vt are eigenvectors; zero beyond S1)
__global__ void first_core_kernel(const double* Vt, int64_t S1, int64_t r0, int64_t r1, double* core) {
  const int64_t n = r0 * S1 * r1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a1 = e % r1, t = e / r1, i = t % S1, a0 = t / S1;
    const int64_t c = a0 * r1 + a1;
    core[e] = c < S1 ? Vt[c * S1 + i] : 0.0;
  }
}

// core_k[a, i, b] = U[a*S + i, b] = Vt[b][a*S + i]
__global__ void mid_core_kernel(const double* Vt, int64_t ra, int64_t S, int64_t rb, int64_t n_eig, double* core) {
  const int64_t n = ra * S * rb;
  const int64_t m = ra * S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % rb, row = e / rb;
    core[e] = b < n_eig ? Vt[b * m + row] : 0.0;
  }
}

// C (r0*r1 x rest) -> C' (r1, rest, r0): C'[a1, x, a0] = C[a0*r1 + a1, x]
__global__ void move_first_last_kernel(const double* C, int64_t r0, int64_t r1, int64_t rest, double* out) {
  const int64_t n = r0 * r1 * rest;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = e % r0, t = e / r0, x = t % rest, a1 = t / rest;
    out[e] = C[(a0 * r1 + a1) * rest + x];
  }
}

__global__ void trace_minus_kernel(const double* Gram, int64_t m, const double* lam, int64_t keep, double* acc) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double tr = 0.0, kept = 0.0;
  for (int64_t i = 0; i < m; ++i) tr += Gram[i * m + i];
  for (int64_t i = 0; i < keep && i < m; ++i) kept += lam[i];   // eigenvalues of M M^T = sigma^2
  *acc += tr - kept;
}

// X_n[a, i, b] = sum_s U[i, s] core[a, s, b] with U = Ut^T (Ut is S x I)
template <class T>
__global__ void attach_kernel(const double* core, const double* Ut, int64_t ra, int64_t S, int64_t rb, int64_t I,
                              T* out) {
  const int64_t n = ra * I * rb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % rb, t = e / rb, i = t % I, a = t / I;
    double v = 0.0;
    for (int64_t s = 0; s < S; ++s) v = fma(Ut[s * I + i], core[(a * S + s) * rb + b], v);
    out[e] = (T)v;
  }
}

// Squared gap ||G - TR(cores)||^2: each thread reconstructs one entry as
// sum_{a0} (core_1[a0, i1, :] core_2[:, i2, :] ... core_N[:, iN, a0]).
constexpr int MAXR = 64;
struct TRDesc {
  const double* cores[8];
  int64_t S[8];
  int64_t r[9];
  int N;
};

// ||G - TR(G_n)||^2, one entry per thread: the ring's trace for the entry's
// indices, product of the cores' slices from the left, kept in registers
// (RM: the bound on the TR ranks, loops unrolled to it).
template <class T, int RM>
__global__ void gap2_kernel(const T* G, TRDesc d, int64_t total, double* partial) {
  __shared__ double red[16];
  double acc = 0.0;
  const int64_t r0 = d.r[0], r1 = d.r[1];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx[8];
    int64_t t = e;
    for (int k = d.N - 1; k >= 0; --k) {
      idx[k] = t % d.S[k];
      t /= d.S[k];
    }
    double val = 0.0;
    for (int64_t a0 = 0; a0 < r0; ++a0) {
      double v[RM], w[RM];
      const double* c0 = d.cores[0] + (a0 * d.S[0] + idx[0]) * r1;
#pragma unroll
      for (int b = 0; b < RM; ++b) v[b] = b < r1 ? c0[b] : 0.0;
      for (int k = 1; k < d.N; ++k) {
        const int64_t ra = d.r[k], rb = d.r[k + 1], step = d.S[k] * rb;
        const double* c = d.cores[k] + idx[k] * rb;
#pragma unroll
        for (int b = 0; b < RM; ++b) {
          double s = 0.0;
          if (b < rb) {
#pragma unroll
            for (int a = 0; a < RM; ++a)
              if (a < ra) s = fma(v[a], c[a * step + b], s);
          }
          w[b] = s;
        }
#pragma unroll
        for (int b = 0; b < RM; ++b) v[b] = w[b];
      }
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b == a0) val += v[b];
    }
    const double diff = (double)G[e] - val;
    acc = fma(diff, diff, acc);
  }
  acc = warp_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// The partials' sum in a fixed order: one workgroup, strided per thread,
// then across lanes and waves.
__global__ void sum_kernel(const double* partial, int64_t n, double* out) {
  __shared__ double red[16];
  double r = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) r += partial[i];
  r = warp_sum(r);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    *out = s;
  }
}

// Largest remainder of the sweep: r0 r1 x prod_{k>1} S_k after step 1, then
// r_k x prod_{j>k} S_j x r0.
int64_t tr_max_remainder(int N, const int64_t* S, const int64_t* r) {
  int64_t total = 1;
  for (int k = 0; k < N; ++k) total *= S[k];
  int64_t mx = r[0] * r[1] * (total / S[0]);
  int64_t tail = total / S[0];
  for (int k = 1; k < N - 1; ++k) {
    tail /= S[k];
    mx = std::max<int64_t>(mx, r[k + 1] * tail * r[0]);
  }
  return mx;
}

}  // namespace

// workspace: Gd (prod S), two remainder buffers, Gram, lam, Vt, jacobi work
size_t tr_svd_work_bytes(int N, const int64_t* S, const int64_t* r) {
  int64_t total = 1;
  for (int k = 0; k < N; ++k) total *= S[k];
  int64_t maxrem = tr_max_remainder(N, S, r);
  int64_t maxm = S[0];
  for (int k = 1; k < N - 1; ++k) maxm = std::max<int64_t>(maxm, r[k] * S[k]);
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  add((size_t)total * 8);
  add((size_t)maxrem * 8);
  add((size_t)maxrem * 8);
  add((size_t)maxm * maxm * 8);
  add((size_t)maxm * 8);
  add((size_t)maxm * maxm * 8);
  add(std::max(jacobi_work_bytes(maxm), eig_top_ok(maxm, maxm) ? eig_top_work_bytes(maxm, maxm) : (size_t)0));
  return b + 256;
}

hipError_t tr_svd_device(const void* Gcore, int core_elem, int N, const int64_t* S, const int64_t* r,
                         double* const* cores, double* work, size_t, int* info, double* discarded, hipStream_t st) {
  int64_t total = 1;
  for (int k = 0; k < N; ++k) total *= S[k];
  int64_t maxrem = tr_max_remainder(N, S, r);
  int64_t maxm = S[0];
  for (int k = 1; k < N - 1; ++k) maxm = std::max<int64_t>(maxm, r[k] * S[k]);
  char* w = (char*)work;
  auto take = [&](size_t x) { char* p = w; w += (x + 255) & ~(size_t)255; return p; };
  double* Gd = (double*)take((size_t)total * 8);
  double* C1 = (double*)take((size_t)maxrem * 8);
  double* C2 = (double*)take((size_t)maxrem * 8);
  double* Gram = (double*)take((size_t)maxm * maxm * 8);
  double* lam = (double*)take((size_t)maxm * 8);
  double* Vt = (double*)take((size_t)maxm * maxm * 8);
  void* jw = take(std::max(jacobi_work_bytes(maxm), eig_top_ok(maxm, maxm) ? eig_top_work_bytes(maxm, maxm)
                                                                            : (size_t)0));
  hipError_t e;
  // the R leading eigenpairs of the m x m Gram matrix into lam (descending)
  // and the first R rows of Vt (row stride m), signed
  auto leading = [&](int64_t m, int64_t R) -> hipError_t {
    hipError_t r;
    if (eig_top_ok(m, R)) {
      const double* zs[1] = {Gram};
      const int64_t ns[1] = {m}, rs[1] = {R};
      double* ls[1] = {lam};
      double* vs[1] = {Vt};
      void* ws[1] = {jw};
      int* is[1] = {info};
      r = eig_top_batched(1, zs, ns, rs, ls, vs, ws, is, st);
    } else {
      r = jacobi_eig(Gram, m, lam, Vt, jw, info, 40, st);
    }
    if (r != hipSuccess) return r;
    return canonical_sign_rows(Vt, R, m, st);
  };
  if (core_elem == E_F64) hipLaunchKernelGGL(to_double_kernel<double>, dim3(gridn(total)), dim3(256), 0, st, (const double*)Gcore, Gd, total);
  else hipLaunchKernelGGL(to_double_kernel<float>, dim3(gridn(total)), dim3(256), 0, st, (const float*)Gcore, Gd, total);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = fill_zero(discarded, 8, st)) != hipSuccess) return e;

  // step 1
  const int64_t S1 = S[0], rest1 = total / S1, r0r1 = r[0] * r[1];
  if ((e = dgemm(0, 1, S1, S1, rest1, 1.0, Gd, rest1, Gd, rest1, 0.0, Gram, S1, st)) != hipSuccess) return e;
  const int64_t kept1 = std::min<int64_t>(r0r1, S1);
  if ((e = leading(S1, kept1)) != hipSuccess) return e;
  hipLaunchKernelGGL(trace_minus_kernel, dim3(1), dim3(64), 0, st, Gram, S1, lam, r0r1, discarded);
  hipLaunchKernelGGL(first_core_kernel, dim3(gridn(r[0] * S1 * r[1])), dim3(256), 0, st, Vt, S1, r[0], r[1], cores[0]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // remainder C = U_k^T M (r0 r1 x rest1), rows beyond S1 zero
  if ((e = fill_zero(C1, (size_t)r0r1 * rest1 * 8, st)) != hipSuccess) return e;
  if ((e = dgemm(0, 0, kept1, rest1, S1, 1.0, Vt, S1, Gd, rest1, 0.0, C1, rest1, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(move_first_last_kernel, dim3(gridn(r0r1 * rest1)), dim3(256), 0, st, C1, r[0], r[1], rest1, C2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double* cur = C2;
  double* nxt = C1;
  int64_t rest = rest1 * r[0];    // columns of the remainder after moving r0 last (includes S_2..S_N and r0)
  // remainder cur is (r1, S2, ..., SN, r0)
  for (int k = 1; k < N - 1; ++k) {
    const int64_t m = r[k] * S[k];
    const int64_t ncols = (r[k] * rest) / m;   // = prod_{j>k} S_j * r0
    if ((e = dgemm(0, 1, m, m, ncols, 1.0, cur, ncols, cur, ncols, 0.0, Gram, m, st)) != hipSuccess) return e;
    const int64_t keep = std::min<int64_t>(r[k + 1], m);
    if ((e = leading(m, keep)) != hipSuccess) return e;
    hipLaunchKernelGGL(trace_minus_kernel, dim3(1), dim3(64), 0, st, Gram, m, lam, r[k + 1], discarded);
    hipLaunchKernelGGL(mid_core_kernel, dim3(gridn(r[k] * S[k] * r[k + 1])), dim3(256), 0, st, Vt, r[k], S[k],
                       r[k + 1], keep, cores[k]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = fill_zero(nxt, (size_t)r[k + 1] * ncols * 8, st)) != hipSuccess) return e;
    if ((e = dgemm(0, 0, keep, ncols, m, 1.0, Vt, m, cur, ncols, 0.0, nxt, ncols, st)) != hipSuccess) return e;
    std::swap(cur, nxt);
    rest = ncols;
  }
  // last core: (r_{N-1}, S_N, r0)
  const int64_t nlast = r[N - 1] * S[N - 1] * r[0];
  return copy_rows_f64(cores[N - 1], nlast, cur, nlast, 1, nlast, st);
}

hipError_t tr_attach(const double* core, const double* Ut, int64_t ra, int64_t Sn, int64_t rb, int64_t I, void* out,
                     int out_elem, hipStream_t st) {
  const int64_t n = ra * I * rb;
  if (out_elem == E_F64)
    hipLaunchKernelGGL(attach_kernel<double>, dim3(gridn(n)), dim3(256), 0, st, core, Ut, ra, Sn, rb, I, (double*)out);
  else
    hipLaunchKernelGGL(attach_kernel<float>, dim3(gridn(n)), dim3(256), 0, st, core, Ut, ra, Sn, rb, I, (float*)out);
  return hipGetLastError();
}

size_t tr_gap2_work_bytes(int, const int64_t*, const int64_t*) { return 4096 * 8 + 256; }

hipError_t tr_gap2(const void* Gcore, int core_elem, int N, const int64_t* S, const int64_t* r, double* const* cores,
                   double* work, double* out, hipStream_t st) {
  TRDesc d = {};
  d.N = N;
  int64_t total = 1;
  for (int k = 0; k < N; ++k) {
    d.cores[k] = cores[k];
    d.S[k] = S[k];
    total *= S[k];
  }
  for (int k = 0; k <= N; ++k) {
    d.r[k] = r[k];
    if (r[k] > MAXR) return hipErrorInvalidValue;
  }
  const unsigned g = (unsigned)std::min<int64_t>(4096, ceil_div(total, 256));
  int64_t rmax = 1;
  for (int k = 0; k <= N; ++k) rmax = std::max(rmax, r[k]);
#define GAP2(RM)                                                                                                 \
  if (core_elem == E_F64)                                                                                       \
    hipLaunchKernelGGL((gap2_kernel<double, RM>), dim3(g), dim3(256), 0, st, (const double*)Gcore, d, total, work); \
  else                                                                                                          \
    hipLaunchKernelGGL((gap2_kernel<float, RM>), dim3(g), dim3(256), 0, st, (const float*)Gcore, d, total, work)
  if (rmax <= 8) GAP2(8);
  else if (rmax <= 16) GAP2(16);
  else if (rmax <= 32) GAP2(32);
  else GAP2(64);
#undef GAP2
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, st, work, (int64_t)g, out);
  return hipGetLastError();
}

}  // namespace rbki
