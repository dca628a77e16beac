// Small kernels outside the collision path: the normwise difference of two
// right-hand sides per instance (the mixed-precision path against the FP64
// lists kept beside it) and a fill of the inner solvers' clocks.
#include "internal.h"

namespace rtbte {

// Per-instance sums of (a_i - b_i)^2 and b_i^2; grid (nchunk, n_inst), fixed
// summation order: partial[2 (inst nchunk + chunk) + {0, 1}].
__global__ __launch_bounds__(256) void k_diff_norms(const double* __restrict__ a, const double* __restrict__ b,
                                                    const InstInfo* info, double* partial, int nchunk) {
  __shared__ double red[2][4];
  const int inst = blockIdx.y;
  const InstInfo in = info[inst];
  const int64_t n = (int64_t)in.n_el + in.n_ph;
  const int64_t cs = (n + nchunk - 1) / nchunk;
  const int64_t lo = (int64_t)blockIdx.x * cs;
  const int64_t hi = lo + cs < n ? lo + cs : n;
  double d2 = 0.0, b2 = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double bb = b[in.off + i], d = a[in.off + i] - bb;
    d2 += d * d;
    b2 += bb * bb;
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o, 64);
    b2 += __shfl_xor(b2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x / 64] = d2;
    red[1][threadIdx.x / 64] = b2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t k = 2 * ((int64_t)inst * nchunk + blockIdx.x);
    partial[k] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    partial[k + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

hipError_t launch_diff_norms(const double* a, const double* b, const InstInfo* info, double* partial, int n_inst,
                             int nchunk, hipStream_t s) {
  if (n_inst <= 0 || nchunk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diff_norms, dim3(nchunk, n_inst), dim3(256), 0, s, a, b, info, partial, nchunk);
  return hipGetLastError();
}

}  // namespace rtbte

namespace rtbte {

// p[i] = v for i < n (per-instance clocks of the inner solves).
__global__ void k_fill(double* p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace rtbte

namespace rtbte {

// Batched adaptive slow step of MIS: the instances share the slow step, which
// is accepted only when every instance's WRMS error is at most 1, so the
// slow controller is given the largest of the instances' norms.  One thread
// totals each instance's partial sums in chunk order and takes the root of
// their mean (as the controller does), picks the first instance with the
// largest norm (a NaN wins, so a non-finite estimate anywhere fails the
// step) and copies that instance's partial sums and sizes to a one-instance
// slot; the controller, run on that slot, then computes bitwise the norm the
// instance would have alone.
__global__ void k_select_max_norm(const double* partial, const InstInfo* info, int n_inst, int nchunk,
                                  double* sel_partial, InstInfo* sel_info) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int best = 0;
  double best_e = -1.0;
  for (int i = 0; i < n_inst; ++i) {
    double s = 0.0;
    for (int j = 0; j < nchunk; ++j) s += partial[(int64_t)i * nchunk + j];
    const double e = sqrt(s / (double)((int64_t)info[i].n_el + info[i].n_ph));
    if (isnan(e)) {
      best = i;
      break;
    }
    if (e > best_e) {
      best_e = e;
      best = i;
    }
  }
  for (int j = 0; j < nchunk; ++j) sel_partial[j] = partial[(int64_t)best * nchunk + j];
  *sel_info = info[best];
}

hipError_t launch_select_max_norm(const double* partial, const InstInfo* info, int n_inst, int nchunk,
                                  double* sel_partial, InstInfo* sel_info, hipStream_t s) {
  if (n_inst <= 0 || nchunk <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select_max_norm, dim3(1), dim3(64), 0, s, partial, info, n_inst, nchunk, sel_partial,
                     sel_info);
  return hipGetLastError();
}

// p[i] = p[0] for 0 < i < n (a common value handed to every instance).
__global__ void k_broadcast_first(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > 0 && i < n) p[i] = p[0];
}

hipError_t launch_broadcast_first(double* p, int64_t n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_broadcast_first, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace rtbte
