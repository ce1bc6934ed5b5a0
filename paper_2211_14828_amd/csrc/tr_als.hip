// TR-ALS of the small Tucker core (Alg. 3, step 3), float64 on the device.
//
// With cores Z_1..Z_N (Z_j is r_{j-1} x S_j x r_j, r_0 = r_N) the ring's
// entries are T(i_1..i_N) = Tr(Z_k(i_k) Z_{k+1}(i_{k+1}) ... Z_{k-1}(i_{k-1}))
// for every k, so with the other cores fixed the model is linear in Z_k:
//   T_<k>[i_k, p] = sum_{a, b} Z_k[a, i_k, b] M[b, p, a],
// M = Z_{k+1} ... Z_N Z_1 ... Z_{k-1} (r_k x P x r_{k-1}), p running over the
// other modes in cyclic order from k+1.  One update of core k solves the
// least-squares problem G_<k> ~ Z_k D^T with the design matrix
// D[p, a r_k + b] = M[b, p, a], by the normal equations A = D^T D,
// equilibrated by A's diagonal, solved with the pseudo-inverse from the
// eigenpairs (eigenvalues below 1e-13 of the largest count as zero, so
// directions that D does not reach, such as the zero-padded ranks of a TR-SVD
// start, keep coefficient zero), and refined twice on the least-squares
// residual.  A sweep updates k = 1..N;
// after it the Fit 1 - ||G - TR|| / ||G|| comes from the last update's
// residual, and the iteration stops when it changes by at most fit_tol
// (the rule of Sec. 4), or after max_sweeps sweeps.  The cores start from
// Gaussian values of the sketch stream (tag 2), scaled by
// 1/sqrt(S_k r_{k-1} r_k): a zero-padded TR-SVD start would make the updates
// rank-deficient.
//
// Every product is a float64 GEMM of linalg.hip; the reductions run in a
// fixed order, so results are deterministic.
#include "rbki_kernels.h"
#include "rbki_philox.h"

namespace rbki {

hipError_t tr_gap2(const void* Gcore, int core_elem, int N, const int64_t* S, const int64_t* r, double* const* cores,
                   double* work, double* out, hipStream_t st);
size_t tr_gap2_work_bytes(int N, const int64_t* S, const int64_t* r);

namespace {

inline unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 8192)); }

// out = G with its axes in the order k, k+1, ..., N-1, 0, ..., k-1
struct Perm {
  int64_t S[8];
  int N, k;
};
__global__ void cyclic_unfold_kernel(const double* __restrict__ G, Perm pm, int64_t total, double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    // e enumerates out in row-major order over the permuted axes
    int64_t t = e, src = 0, idx[8];
    for (int j = pm.N - 1; j >= 0; --j) {
      const int ax = (pm.k + j) % pm.N;
      idx[ax] = t % pm.S[ax];
      t /= pm.S[ax];
    }
    for (int ax = 0; ax < pm.N; ++ax) src = src * pm.S[ax] + idx[ax];
    out[e] = G[src];
  }
}

// The start: core k's entry at linear index L is the Gaussian z(L) of the
// sketch stream (seed, k, tag 2) divided by sqrt(S_k r_{k-1} r_k).
constexpr uint32_t TAG_TR_START = 2;
__global__ void start_core_kernel(double* __restrict__ core, int64_t n, uint32_t k, uint64_t seed, double scale) {
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n; L += (int64_t)gridDim.x * blockDim.x) {
    double ze, zo;
    gauss_pair_f64((uint64_t)L >> 1, k, TAG_TR_START, seed, ze, zo);
    core[L] = ((L & 1) ? zo : ze) * scale;
  }
}

// D[p, a rk + b] = M[b, p, a] with M of shape (rk, P, rk1)
__global__ void design_kernel(const double* __restrict__ M, int64_t rk, int64_t P, int64_t rk1, double* __restrict__ D) {
  const int64_t total = P * rk1 * rk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % rk, t = e / rk, a = t % rk1, p = t / rk1;
    D[e] = M[(b * P + p) * rk1 + a];
  }
}

// column equilibration of the normal equations: sc[i] = 1 / sqrt(A_ii)
// (1 for a zero column), then A_ij <- sc_i A_ij sc_j (one workgroup)
__global__ void equilibrate_kernel(double* __restrict__ A, int64_t n, double* __restrict__ sc) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = A[i * n + i];
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < n * n; e += blockDim.x) A[e] *= sc[e / n] * sc[e % n];
}

// M[i, :] *= sc[i]
__global__ void scale_rows_kernel(double* __restrict__ M, const double* __restrict__ sc, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    M[e] *= sc[e / cols];
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void add_kernel(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] += src[e];
}

// rows j of T scaled by 1 / lam[j] where lam[j] > thr * lam[0], else zeroed
__global__ void pinv_scale_kernel(double* __restrict__ T, const double* __restrict__ lam, int64_t n, int64_t cols) {
  const double thr = 1e-13 * lam[0];
  const int64_t total = n * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const double l = lam[e / cols];
    T[e] = l > thr ? T[e] / l : 0.0;
  }
}

// core[a, i, b] = Xc[a rk + b, i]
__global__ void coeffs_to_core_kernel(const double* __restrict__ Xc, int64_t rk1, int64_t S, int64_t rk,
                                      double* __restrict__ core) {
  const int64_t total = rk1 * S * rk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % rk, t = e / rk, i = t % S, a = t / S;
    core[e] = Xc[(a * rk + b) * S + i];
  }
}

// partial[block] = sum over its share of (x - y)^2 (y null: x^2); then one
// fixed-order sum
__global__ void sumsq_diff_kernel(const double* __restrict__ x, const double* __restrict__ y, int64_t n,
                                  double* __restrict__ partial) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double d = y ? x[e] - y[e] : x[e];
    acc = fma(d, d, acc);
  }
  acc = warp_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void sum_partials_kernel(const double* __restrict__ partial, int64_t n, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += partial[i];
  *out = s;
}

struct AlsSizes {
  int64_t total = 1, maxM = 0, maxD = 0, maxR2 = 0, maxS = 0;
};

AlsSizes als_sizes(int N, const int64_t* S, const int64_t* r) {
  AlsSizes z;
  for (int k = 0; k < N; ++k) {
    z.total *= S[k];
    z.maxS = std::max(z.maxS, S[k]);
  }
  for (int k = 0; k < N; ++k) {
    // the product Z_{k+1} ... Z_{k+j} holds r_{k+1} x (their S) x r_{k+j+1}
    // values (ranks indexed as in r[0..N])
    const int o1 = (k + 1) % N;
    int64_t prodS = S[o1];
    for (int j = 2; j < N; ++j) {
      const int o = (k + j) % N;
      prodS *= S[o];
      z.maxM = std::max(z.maxM, r[o1] * prodS * r[o + 1]);
    }
    z.maxD = std::max(z.maxD, (z.total / S[k]) * r[k] * r[k + 1]);
    z.maxR2 = std::max(z.maxR2, r[k] * r[k + 1]);
  }
  z.maxM = std::max<int64_t>(z.maxM, 1);
  return z;
}

constexpr int64_t kPartials = 1024;

}  // namespace

size_t tr_als_work_bytes(int N, const int64_t* S, const int64_t* r) {
  const AlsSizes z = als_sizes(N, S, r);
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  add((size_t)z.maxM * 8);           // two buffers of the growing product
  add((size_t)z.maxM * 8);
  add((size_t)z.maxD * 8);           // D
  add((size_t)z.total * 8);          // G_<k>
  add((size_t)z.total * 8);          // the model's G_<k>
  add((size_t)z.maxR2 * z.maxR2 * 8);    // A, its eigenvectors
  add((size_t)z.maxR2 * z.maxR2 * 8);
  add((size_t)z.maxR2 * 8);          // eigenvalues
  add((size_t)z.maxR2 * z.maxS * 8);     // B, T, the coefficients
  add((size_t)z.maxR2 * z.maxS * 8);
  add((size_t)z.maxR2 * z.maxS * 8);
  add((size_t)z.maxR2 * 8);          // column scales
  add(jacobi_work_bytes(z.maxR2));
  add(kPartials * 8 + 64);
  add(tr_gap2_work_bytes(N, S, r));
  return b + 256;
}

// Gd: the core (prod S) in float64; cores: N device pointers that receive
// the start and then the result; r[0..N] with r[0] = r[N].  info: device ints (Jacobi sweep-limit flag).  *sweeps_out and
// *err2_out (host): the sweeps taken and ||G - TR||^2 after the last one.
hipError_t tr_als_device(const double* Gd, int N, const int64_t* S, const int64_t* r, double* const* cores,
                         uint64_t seed, int max_sweeps, double fit_tol, void* work, int* info, int* sweeps_out,
                         double* err2_out, hipStream_t st) {
  const AlsSizes z = als_sizes(N, S, r);
  char* w = (char*)work;
  auto take = [&](size_t x) { char* p = w; w += (x + 255) & ~(size_t)255; return p; };
  double* M0 = (double*)take((size_t)z.maxM * 8);
  double* M1 = (double*)take((size_t)z.maxM * 8);
  double* D = (double*)take((size_t)z.maxD * 8);
  double* Gk = (double*)take((size_t)z.total * 8);
  double* Mk = (double*)take((size_t)z.total * 8);
  double* A = (double*)take((size_t)z.maxR2 * z.maxR2 * 8);
  double* Vt = (double*)take((size_t)z.maxR2 * z.maxR2 * 8);
  double* lam = (double*)take((size_t)z.maxR2 * 8);
  double* B = (double*)take((size_t)z.maxR2 * z.maxS * 8);
  double* T = (double*)take((size_t)z.maxR2 * z.maxS * 8);
  double* Zc = (double*)take((size_t)z.maxR2 * z.maxS * 8);
  double* sc = (double*)take((size_t)z.maxR2 * 8);
  void* jw = take(jacobi_work_bytes(z.maxR2));
  double* part = (double*)take(kPartials * 8 + 64);
  double* red = part + kPartials;
  double* gw = (double*)take(tr_gap2_work_bytes(N, S, r));
  hipError_t e;

  // the start, its error (the reference of the first Fit change), ||G||^2
  for (int k = 0; k < N; ++k) {
    const int64_t n = r[k] * S[k] * r[k + 1];
    hipLaunchKernelGGL(start_core_kernel, dim3(grid_of(n)), dim3(256), 0, st, cores[k], n, (uint32_t)k, seed,
                       1.0 / std::sqrt((double)n));
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double h0 = 0.0, g2 = 0.0;
  if ((e = tr_gap2(Gd, E_F64, N, S, r, cores, gw, red, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&h0, red, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  const unsigned pg = (unsigned)std::min<int64_t>(kPartials, ceil_div(z.total, 256));
  hipLaunchKernelGGL(sumsq_diff_kernel, dim3(pg), dim3(256), 0, st, Gd, (const double*)nullptr, z.total, part);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, (const double*)part, (int64_t)pg, red + 1);
  if ((e = hipMemcpyAsync(&g2, red + 1, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  const double gn = std::sqrt(g2);
  double prev = gn > 0.0 ? 1.0 - std::sqrt(h0) / gn : 1.0;
  double err2 = h0;
  int sweeps = 0;
  for (int sw = 1; sw <= max_sweeps; ++sw) {
    sweeps = sw;
    for (int k = 0; k < N; ++k) {
      const int64_t rk1 = r[k], rk = r[k + 1], Sk = S[k], P = z.total / Sk, n2 = rk1 * rk;
      // M = Z_{k+1} ... Z_{k-1}: (rows, r) x (r, S r') products
      int o = (k + 1) % N;
      const double* cur = cores[o];
      int64_t rows = r[o] * S[o];          // rows of the product so far, the right rank in columns
      int64_t rc = r[o + 1];
      double* bufs[2] = {M0, M1};
      int wb = 0;
      for (int j = 2; j < N; ++j) {
        o = (k + j) % N;
        double* dst = bufs[wb];
        if ((e = dgemm(0, 0, rows, S[o] * r[o + 1], rc, 1.0, cur, rc, cores[o], S[o] * r[o + 1], 0.0, dst,
                       S[o] * r[o + 1], st)) != hipSuccess)
          return e;
        rows *= S[o];
        rc = r[o + 1];
        cur = dst;
        wb ^= 1;
      }
      // cur is (r_k, P, r_{k-1}); the design matrix and G_<k>
      hipLaunchKernelGGL(design_kernel, dim3(grid_of(P * n2)), dim3(256), 0, st, cur, rk, P, rk1, D);
      Perm pm = {};
      pm.N = N;
      pm.k = k;
      for (int j = 0; j < N; ++j) pm.S[j] = S[j];
      hipLaunchKernelGGL(cyclic_unfold_kernel, dim3(grid_of(z.total)), dim3(256), 0, st, Gd, pm, z.total, Gk);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      // normal equations, equilibrated (A_s = Sc A Sc with Sc = diag(A)^-1/2),
      // the pseudo-inverse of A_s from its eigenpairs, and two steps of
      // iterative refinement on the least-squares residual, which recover
      // the accuracy that forming D^T D loses
      if ((e = dgemm(1, 0, n2, n2, P, 1.0, D, n2, D, n2, 0.0, A, n2, st)) != hipSuccess) return e;
      hipLaunchKernelGGL(equilibrate_kernel, dim3(1), dim3(256), 0, st, A, n2, sc);
      if ((e = jacobi_eig(A, n2, lam, Vt, jw, info, 40, st)) != hipSuccess) return e;
      const double* R = Gk;                // the residual G_<k> - Zc^T D^T, transposed (S_k x P)
      for (int it = 0; it < 3; ++it) {
        // correction Sc A_s^+ Sc D^T R^T
        if ((e = dgemm(1, 1, n2, Sk, P, 1.0, D, n2, R, P, 0.0, B, Sk, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_of(n2 * Sk)), dim3(256), 0, st, B, (const double*)sc, n2, Sk);
        if ((e = dgemm(0, 0, n2, Sk, n2, 1.0, Vt, n2, B, Sk, 0.0, T, Sk, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(pinv_scale_kernel, dim3(grid_of(n2 * Sk)), dim3(256), 0, st, T, (const double*)lam, n2,
                           Sk);
        if ((e = dgemm(1, 0, n2, Sk, n2, 1.0, Vt, n2, T, Sk, 0.0, it == 0 ? Zc : B, Sk, st)) != hipSuccess) return e;
        if (it == 0) {
          hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_of(n2 * Sk)), dim3(256), 0, st, Zc, (const double*)sc, n2,
                             Sk);
        } else {
          hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_of(n2 * Sk)), dim3(256), 0, st, B, (const double*)sc, n2,
                             Sk);
          hipLaunchKernelGGL(add_kernel, dim3(grid_of(n2 * Sk)), dim3(256), 0, st, Zc, (const double*)B, n2 * Sk);
        }
        hipLaunchKernelGGL(copy_kernel, dim3(grid_of(z.total)), dim3(256), 0, st, Mk, (const double*)Gk, z.total);
        if ((e = dgemm(1, 1, Sk, P, n2, -1.0, Zc, Sk, D, n2, 1.0, Mk, P, st)) != hipSuccess) return e;
        R = Mk;
      }
      hipLaunchKernelGGL(coeffs_to_core_kernel, dim3(grid_of(n2 * Sk)), dim3(256), 0, st, (const double*)Zc, rk1,
                         Sk, rk, cores[k]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (k == N - 1) {
        // the Fit after the sweep: the last update's residual
        hipLaunchKernelGGL(sumsq_diff_kernel, dim3(pg), dim3(256), 0, st, (const double*)Mk, (const double*)nullptr,
                           z.total, part);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, (const double*)part, (int64_t)pg, red);
        if ((e = hipMemcpyAsync(&err2, red, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
      }
    }
    const double fit = gn > 0.0 ? 1.0 - std::sqrt(err2) / gn : 1.0;
    if (std::fabs(fit - prev) <= fit_tol) break;
    prev = fit;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (err2_out) *err2_out = err2;
  return hipSuccess;
}

}  // namespace rbki
