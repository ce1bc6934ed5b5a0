// Partial-column sampling of a mode unfolding (Sec. 3.1: the block Krylov
// space may be built from a fraction omega of the columns of X_(n)).
//
// The sample is stratified and uniform: the J columns are split into m
// consecutive strata [floor(k J / m), floor((k+1) J / m)) and stratum k
// contributes the column at offset floor(w width / 2^32), with w the first
// output word of the Philox4x32-10 block at counter (lo32(k), hi32(k), mode,
// tag 1) under the sketch key.  Integer arithmetic only, so every thread
// finds its column on its own and the m columns come out in increasing order.
//
// The gather reads the sampled columns of the view [A, I, B] (column
// j = a B + b is the fibre X[a, :, b]) into a row-major I x m matrix, which the
// Gram / sketch kernels then read as the view [1, I, m].
#include "rbki_kernels.h"
#include "rbki_philox.h"

namespace rbki {

namespace {

constexpr uint32_t TAG_COLUMNS = 1;

__global__ void sample_columns_kernel(uint64_t seed, uint32_t mode, uint64_t J, uint64_t m, int64_t* cols) {
  for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < m; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = k * J / m;
    const uint64_t width = (k + 1) * J / m - lo;
    const PhiloxOut o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), mode, TAG_COLUMNS, (uint32_t)seed,
                                      (uint32_t)(seed >> 32));
    cols[k] = (int64_t)(lo + (((uint64_t)o.w0 * width) >> 32));
  }
}

template <class T> __device__ inline float load_as_float(const T* p);
template <> __device__ inline float load_as_float<float>(const float* p) { return *p; }
template <> __device__ inline float load_as_float<double>(const double* p) { return (float)*p; }
template <> __device__ inline float load_as_float<bf16_t>(const bf16_t* p) { return bf16_to_f32(*p); }

// Y[i, k] = X[a_k, i, b_k]: each workgroup takes 256 consecutive samples of
// one row block; the column indices are read once per thread and reused for
// its rows.
template <class TI, class TO>
__global__ void gather_columns_kernel(const TI* __restrict__ X, int64_t I, int64_t B, const int64_t* __restrict__ cols,
                                      int64_t m, TO* __restrict__ Y) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t c = cols[k];
  const int64_t a = c / B, b = c - a * B;
  const TI* src = X + (a * I) * B + b;
  const int64_t i0 = (int64_t)blockIdx.y * 16;
  const int64_t i1 = i0 + 16 < I ? i0 + 16 : I;
  for (int64_t i = i0; i < i1; ++i) {
    if constexpr (sizeof(TO) == 2 && sizeof(TI) != 2) {
      Y[i * m + k] = f32_to_bf16(load_as_float<TI>(src + i * B));
    } else {
      Y[i * m + k] = src[i * B];
    }
  }
}

template <class TI, class TO>
hipError_t gather_t(const void* X, int64_t I, int64_t B, const int64_t* cols, int64_t m, void* Y, hipStream_t s) {
  const dim3 grid((unsigned)ceil_div(m, 256), (unsigned)ceil_div(I, 16));
  hipLaunchKernelGGL((gather_columns_kernel<TI, TO>), grid, dim3(256), 0, s, (const TI*)X, I, B, cols, m, (TO*)Y);
  return hipGetLastError();
}

}  // namespace

int64_t sample_count(int64_t J, double rate) {
  if (!(rate < 1.0)) return J;
  const double v = floor(rate * (double)J + 0.5);
  return std::max<int64_t>(1, std::min<int64_t>(J, (int64_t)v));
}

hipError_t launch_sample_columns(uint64_t seed, int mode, int64_t J, int64_t m, int64_t* cols, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(m, 256), 4096);
  hipLaunchKernelGGL(sample_columns_kernel, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, (uint64_t)J,
                     (uint64_t)m, cols);
  return hipGetLastError();
}

hipError_t launch_gather_columns(int x_elem, const void* X, int64_t I, int64_t B, const int64_t* cols, int64_t m,
                                 int y_elem, void* Y, hipStream_t s) {
  if (m <= 0 || I <= 0) return hipSuccess;
  if (ceil_div(I, 16) > 65535) return hipErrorInvalidValue;
  if (y_elem == x_elem) {
    if (x_elem == E_F64) return gather_t<double, double>(X, I, B, cols, m, Y, s);
    if (x_elem == E_F32) return gather_t<float, float>(X, I, B, cols, m, Y, s);
    if (x_elem == E_BF16) return gather_t<bf16_t, bf16_t>(X, I, B, cols, m, Y, s);
    return hipErrorInvalidValue;
  }
  if (y_elem != E_BF16) return hipErrorInvalidValue;
  if (x_elem == E_F64) return gather_t<double, bf16_t>(X, I, B, cols, m, Y, s);
  if (x_elem == E_F32) return gather_t<float, bf16_t>(X, I, B, cols, m, Y, s);
  return hipErrorInvalidValue;
}

}  // namespace rbki
