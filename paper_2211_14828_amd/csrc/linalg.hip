// Float64 dense linear algebra on small matrices (the Krylov basis, the
// projected matrix Z and its eigenvectors).  Every routine here works on
// matrices of at most a few thousand rows/columns and runs entirely on the
// device.
#include <hip/hip_cooperative_groups.h>

#include "rbki_kernels.h"

namespace cg = cooperative_groups;

namespace rbki {

namespace {

// ------------------------------------------------------------------ DGEMM
// 64 x 64 output tile per 256-thread workgroup, 4 x 4 outputs per thread,
// K staged through LDS in steps of 16.
constexpr int GT = 64, GK = 16;

__global__ void __launch_bounds__(256) dgemm_kernel(int opA, int opB, int64_t m, int64_t n, int64_t k,
                                                    double alpha, const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb, double beta,
                                                    double* __restrict__ C, int64_t ldc) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t row0 = (int64_t)blockIdx.y * GT, col0 = (int64_t)blockIdx.x * GT;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < k; k0 += GK) {
    // stage A tile: As[kk][i] = op(A)[row0 + i, k0 + kk]
    for (int e = threadIdx.x; e < GK * GT; e += 256) {
      int kk, i;
      if (opA == 0) { i = e / GK; kk = e % GK; } else { kk = e / GT; i = e % GT; }
      const int64_t r = row0 + i, c = k0 + kk;
      double v = 0.0;
      if (r < m && c < k) v = opA == 0 ? A[r * lda + c] : A[c * lda + r];
      As[kk][i] = v;
    }
    for (int e = threadIdx.x; e < GK * GT; e += 256) {
      int kk, j;
      if (opB == 0) { kk = e / GT; j = e % GT; } else { j = e / GK; kk = e % GK; }
      const int64_t r = k0 + kk, c = col0 + j;
      double v = 0.0;
      if (r < k && c < n) v = opB == 0 ? B[r * ldb + c] : B[c * ldb + r];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty + 16 * u];
        b[u] = Bs[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = row0 + ty + 16 * u, c = col0 + tx + 16 * v;
      if (r < m && c < n) {
        double* p = C + r * ldc + c;
        *p = beta == 0.0 ? alpha * acc[u][v] : alpha * acc[u][v] + beta * *p;
      }
    }
}

// ------------------------------------------------------------ Cholesky QR
// Left-looking Cholesky of the s x s Gram matrix G with column dropping, one
// workgroup.  A pivot d_k = G_kk - sum_j L_kj^2 is dropped (column of L set
// to zero) when d_k <= tau_rel * G_kk (the vector lies within the span of the
// earlier kept ones to working accuracy) or d_k <= tau_abs^2 * max_k ref2[k]
// (it is at round-off level relative to the block before projection).
__global__ void __launch_bounds__(1024) chol_drop_kernel(const double* G, int64_t s, double* L, int* flags,
                                                         const double* ref2, double tau_rel, double tau_abs) {
  __shared__ double red[16];
  __shared__ double sh_ref;
  __shared__ int sh_keep;
  __shared__ double sh_piv;
  const int tid = threadIdx.x;
  // max reference norm
  double mx = 0.0;
  if (ref2)
    for (int64_t i = tid; i < s; i += blockDim.x) mx = fmax(mx, ref2[i]);
  mx = warp_max(mx);
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
    sh_ref = v;
  }
  for (int64_t i = tid; i < s * s; i += blockDim.x) L[i] = 0.0;
  __syncthreads();
  const double abs_floor = tau_abs * tau_abs * sh_ref;
  for (int64_t kc = 0; kc < s; ++kc) {
    if (tid == 0) {
      double d = G[kc * s + kc];
      for (int64_t j = 0; j < kc; ++j) d -= L[kc * s + j] * L[kc * s + j];
      const double gkk = G[kc * s + kc];
      const int keep = (gkk > 0.0) && (d > tau_rel * gkk) && (d > abs_floor);
      sh_keep = keep;
      sh_piv = keep ? sqrt(d) : 0.0;
      flags[kc] = keep;
      if (keep) L[kc * s + kc] = sh_piv;
    }
    __syncthreads();
    if (sh_keep) {
      const double piv = sh_piv;
      for (int64_t i = kc + 1 + tid; i < s; i += blockDim.x) {
        double v = G[i * s + kc];
        for (int64_t j = 0; j < kc; ++j) v -= L[i * s + j] * L[kc * s + j];
        L[i * s + kc] = v / piv;
      }
    }
    __syncthreads();
  }
}

// Y (s x n rows) <- L^{-1} Y row-wise (forward substitution along the s
// vectors), one thread per column; dropped vectors become zero.
__global__ void trsm_rows_kernel(double* Y, int64_t s, int64_t n, const double* L, const int* flags) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t kc = 0; kc < s; ++kc) {
      if (!flags[kc]) {
        Y[kc * n + c] = 0.0;
        continue;
      }
      double v = Y[kc * n + c];
      for (int64_t j = 0; j < kc; ++j)
        if (flags[j]) v -= L[kc * s + j] * Y[j * n + c];
      Y[kc * n + c] = v / L[kc * s + kc];
    }
  }
}

__global__ void row_norms2_kernel(const double* Y, int64_t s, int64_t n, double* out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= s) return;
  double acc = 0.0;
  for (int64_t c = lane; c < n; c += 64) {
    const double v = Y[row * n + c];
    acc = fma(v, v, acc);
  }
  acc = warp_sum(acc);
  if (lane == 0) out[row] = acc;
}

// ------------------------------------------------------------ Jacobi
// Block one-sided (Hestenes) Jacobi on the columns of a symmetric PSD matrix.
// The n columns are split into nblk blocks of nb columns (zero-padded).
// Rounds follow the circle method over blocks: in each round every
// workgroup takes one pair of blocks, stages their 2*nb columns in LDS, and
// orthogonalises every pair of those columns once (an inner cyclic sweep).
// nblk - 1 rounds make one sweep; all workgroups meet at a grid barrier
// between rounds.  The sweep ends the iteration when no pair needed a
// rotation above tol (largest |cos| between two columns).  At convergence
// A = Z V has orthogonal columns a_j = lambda_j v_j, so the eigenvalues are
// the column norms and the eigenvectors the normalised columns.
struct JacobiArgs {
  double* A;        // npad x n column-major working copy (column j at A + j*n)
  int64_t n, npad;
  int nb, nblk;
  int max_sweeps;
  double tol;
  unsigned long long* offmax;   // [3] per-sweep max |cos| bit patterns (rotating slots)
  int* info;
};

__device__ inline int circle_block(int pos, int round, int nblk) {
  if (pos == 0) return 0;
  return 1 + (pos - 1 + round) % (nblk - 1);
}

__global__ void __launch_bounds__(1024) jacobi_kernel(JacobiArgs J) {
  extern __shared__ double cols[];               // 2*nb columns of length n
  __shared__ double sh_off[16];
  __shared__ int sh_stop;
  cg::grid_group grid = cg::this_grid();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int64_t n = J.n;
  const int nb = J.nb, two = 2 * nb;
  int sweep;
  for (sweep = 0; sweep < J.max_sweeps; ++sweep) {
    // slot sweep%3 collects this sweep; slot (sweep+1)%3 was last read two
    // grid barriers ago and is cleared for the next sweep
    if (blockIdx.x == 0 && tid == 0) J.offmax[(sweep + 1) % 3] = 0ull;
    double local_off = 0.0;
    for (int round = 0; round < J.nblk - 1; ++round) {
      const int pos = blockIdx.x;
      const int bp = circle_block(pos, round, J.nblk);
      const int bq = circle_block(J.nblk - 1 - pos, round, J.nblk);
      // stage: local column c < nb from block bp, else from bq
      for (int64_t e = tid; e < (int64_t)two * n; e += blockDim.x) {
        const int c = (int)(e / n);
        const int64_t r = e - (int64_t)c * n;
        const int gc = (c < nb ? bp * nb + c : bq * nb + (c - nb));
        cols[e] = J.A[(int64_t)gc * n + r];
      }
      __syncthreads();
      // inner cyclic sweep over the 2nb local columns (circle method again)
      for (int ir = 0; ir < two - 1; ++ir) {
        for (int pr = wave; pr < nb; pr += nwaves) {
          const int p = circle_block(pr, ir, two);
          const int q = circle_block(two - 1 - pr, ir, two);
          double* cp = cols + (int64_t)p * n;
          double* cq = cols + (int64_t)q * n;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int64_t r = lane; r < n; r += 64) {
            const double x = cp[r], y = cq[r];
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
          al = warp_sum(al);
          be = warp_sum(be);
          ga = warp_sum(ga);
          const double nrm = sqrt(al) * sqrt(be);
          if (nrm > 1e-300) {
            const double cosang = fabs(ga) / nrm;
            local_off = fmax(local_off, cosang);
            if (cosang > J.tol) {
              const double zeta = (be - al) / (2.0 * ga);
              const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
              for (int64_t r = lane; r < n; r += 64) {
                const double x = cp[r], y = cq[r];
                cp[r] = c * x - s * y;
                cq[r] = s * x + c * y;
              }
            }
          }
        }
        __syncthreads();
      }
      for (int64_t e = tid; e < (int64_t)two * n; e += blockDim.x) {
        const int c = (int)(e / n);
        const int64_t r = e - (int64_t)c * n;
        const int gc = (c < nb ? bp * nb + c : bq * nb + (c - nb));
        J.A[(int64_t)gc * n + r] = cols[e];
      }
      __threadfence();
      grid.sync();
    }
    // publish this workgroup's largest |cos| of the sweep
    local_off = warp_max(local_off);
    if (lane == 0) sh_off[wave] = local_off;
    __syncthreads();
    if (tid == 0) {
      double v = 0.0;
      for (int w = 0; w < nwaves; ++w) v = fmax(v, sh_off[w]);
      atomicMax(&J.offmax[sweep % 3], (unsigned long long)__double_as_longlong(v));
    }
    __threadfence();
    grid.sync();
    if (tid == 0) {
      const double v = __longlong_as_double((long long)__atomic_load_n(&J.offmax[sweep % 3], __ATOMIC_RELAXED));
      sh_stop = v <= J.tol;
    }
    __syncthreads();
    if (sh_stop) break;
  }
  if (blockIdx.x == 0 && tid == 0) *J.info = (sweep >= J.max_sweeps) ? sweep : 0;
}

// Column norms of the converged A, then a rank sort (descending, ties by
// index) and normalised columns as rows of Vt.
__global__ void jacobi_finish_kernel(const double* A, int64_t n, double* lam, double* Vt, double* norms) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  for (int64_t j = wave; j < n; j += nwaves) {
    double acc = 0.0;
    for (int64_t r = lane; r < n; r += 64) acc = fma(A[j * n + r], A[j * n + r], acc);
    acc = warp_sum(acc);
    if (lane == 0) norms[j] = sqrt(acc);
  }
  __syncthreads();
  for (int64_t j = tid; j < n; j += blockDim.x) {
    const double v = norms[j];
    int64_t rank = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double w = norms[i];
      rank += (w > v) || (w == v && i < j);
    }
    lam[rank] = v;
    // stash the destination row in the sign-free slot: handled below
    norms[n + j] = (double)rank;
  }
  __syncthreads();
  for (int64_t e = tid; e < n * n; e += blockDim.x) {
    const int64_t j = e / n, r = e - j * n;
    const int64_t dst = (int64_t)norms[n + j];
    const double nv = norms[j];
    Vt[dst * n + r] = nv > 0.0 ? A[j * n + r] / nv : 0.0;
  }
}

__global__ void pad_copy_kernel(const double* Z, int64_t n, int64_t npad, double* A) {
  // A column-major n x npad: column j = row j of Z (Z symmetric), zero beyond n
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npad * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / n, r = e - j * n;
    A[e] = j < n ? Z[j * n + r] : 0.0;
  }
}

__global__ void copy_rows_kernel(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows,
                                 int64_t cols) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

template <class T>
__global__ void store_factor_kernel(const double* Ut, int64_t R, int64_t I, T* out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < R * I;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R, r = e - i * R;
    out[e] = (T)Ut[r * I + i];
  }
}

// Sign rule for singular/eigen vectors: flip each row of V (rows x n) so that
// its largest-magnitude entry (lowest index on ties) is positive.  One wave per row.
__global__ void canonical_sign_rows_kernel(double* V, int64_t rows, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= rows) return;
  double* v = V + row * n;
  double best = -1.0;
  int64_t bi = n;
  for (int64_t c = lane; c < n; c += 64) {
    const double a = fabs(v[c]);
    if (a > best) { best = a; bi = c; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if (best <= 0.0 || bi >= n) return;
  const double sgn = v[bi] < 0.0 ? -1.0 : 1.0;
  if (sgn < 0.0)
    for (int64_t c = lane; c < n; c += 64) v[c] = -v[c];
}

__global__ void fill_zero_kernel(unsigned* p, size_t words) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < words; e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

inline unsigned grid_for(int64_t work, int64_t per = 256, int64_t cap = 8192) {
  int64_t g = ceil_div(work, per);
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

}  // namespace

hipError_t dgemm(int opA, int opB, int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)ceil_div(n, GT), (unsigned)ceil_div(m, GT));
  hipLaunchKernelGGL(dgemm_kernel, grid, dim3(256), 0, s, opA, opB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  return hipGetLastError();
}

hipError_t row_norms2(const double* Y, int64_t s, int64_t n, double* out, hipStream_t st) {
  if (s <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_norms2_kernel, dim3((unsigned)ceil_div(s, 4)), dim3(256), 0, st, Y, s, n, out);
  return hipGetLastError();
}

hipError_t chol_orth(double* Y, int64_t s, int64_t n, double* G, double* Lm, int* flags, const double* ref2,
                     double tau_rel, double tau_abs, hipStream_t st) {
  if (s <= 0) return hipSuccess;
  hipError_t e = dgemm(0, 1, s, s, n, 1.0, Y, n, Y, n, 0.0, G, s, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chol_drop_kernel, dim3(1), dim3(1024), 0, st, G, s, Lm, flags, ref2, tau_rel, tau_abs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(trsm_rows_kernel, dim3(grid_for(n)), dim3(256), 0, st, Y, s, n, Lm, flags);
  return hipGetLastError();
}

static void jacobi_geometry(int64_t n, int& nb, int& nblk) {
  nb = n <= 512 ? 16 : 8;
  if (n <= 32) nb = (int)std::max<int64_t>(1, (n + 1) / 2);
  nblk = (int)ceil_div(n, nb);
  if (nblk < 2) nblk = 2;
  if (nblk & 1) ++nblk;
}

size_t jacobi_work_bytes(int64_t n) {
  // npad <= n + 2 * nb <= n + 32, so this bound grows with n and covers every
  // smaller matrix that reuses the same scratch
  return (size_t)((n + 32) * n * 8 + 2 * n * 8 + 64);  // A, norms/ranks, offmax[3]
}

hipError_t jacobi_eig(const double* Z, int64_t n, double* lam, double* Vt, void* work, int* info, int max_sweeps,
                      hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int nb, nblk;
  jacobi_geometry(n, nb, nblk);
  const int64_t npad = (int64_t)nb * nblk;
  char* w = (char*)work;
  double* A = (double*)w;
  double* norms = (double*)(w + npad * n * 8);
  unsigned long long* offmax = (unsigned long long*)(w + npad * n * 8 + 2 * n * 8);
  hipLaunchKernelGGL(pad_copy_kernel, dim3(grid_for(npad * n)), dim3(256), 0, st, Z, n, npad, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, st, (unsigned*)offmax, (size_t)6);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  JacobiArgs ja;
  ja.A = A;
  ja.n = n;
  ja.npad = npad;
  ja.nb = nb;
  ja.nblk = nblk;
  ja.max_sweeps = max_sweeps;
  ja.tol = 1e-13;
  ja.offmax = offmax;
  ja.info = info;
  void* args[] = {&ja};
  const size_t shmem = (size_t)2 * nb * n * 8;
  e = hipFuncSetAttribute((const void*)jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  e = hipLaunchCooperativeKernel((const void*)jacobi_kernel, dim3(nblk / 2), dim3(1024), args, shmem, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(1024), 0, st, A, n, lam, Vt, norms);
  return hipGetLastError();
}

hipError_t copy_rows_f64(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows, int64_t cols,
                         hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_rows_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, st, dst, ldd, src, lds, rows, cols);
  return hipGetLastError();
}

hipError_t store_factor(const double* Ut, int64_t R, int64_t I, void* out, int out_elem, hipStream_t st) {
  if (out_elem == E_F64)
    hipLaunchKernelGGL(store_factor_kernel<double>, dim3(grid_for(R * I)), dim3(256), 0, st, Ut, R, I, (double*)out);
  else
    hipLaunchKernelGGL(store_factor_kernel<float>, dim3(grid_for(R * I)), dim3(256), 0, st, Ut, R, I, (float*)out);
  return hipGetLastError();
}

hipError_t canonical_sign_rows(double* V, int64_t rows, int64_t n, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(canonical_sign_rows_kernel, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, st, V, rows, n);
  return hipGetLastError();
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for((int64_t)(bytes / 4))), dim3(256), 0, st, (unsigned*)p, bytes / 4);
  return hipGetLastError();
}

}  // namespace rbki
