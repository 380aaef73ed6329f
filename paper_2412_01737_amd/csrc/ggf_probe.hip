// Stream probes: a plain copy and an in-place read-modify-write of a large
// buffer, with and without non-temporal hints.  They calibrate the HBM traffic
// counters and give the achievable bandwidth the rank-4 update is compared with.
#include <hip/hip_runtime.h>

#include "ggf_launch.h"

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));

template <bool NT>
__global__ __launch_bounds__(256) void k_probe_copy(const d2v *__restrict__ src, d2v *__restrict__ dst,
                                                    size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    else dst[i] = src[i];
  }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_probe_rmw(d2v *__restrict__ a, size_t n, double s) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    d2v v = NT ? __builtin_nontemporal_load(a + i) : a[i];
    v.x = fma(v.x, s, 1.0);
    v.y = fma(v.y, s, 1.0);
    if (NT) __builtin_nontemporal_store(v, a + i);
    else a[i] = v;
  }
}

}  // namespace

int ggf_launch_probe(int mode, void *a, void *b, size_t bytes, int grid, hipStream_t s) {
  const size_t n = bytes / sizeof(double2);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe_copy<false>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    case 1: hipLaunchKernelGGL(k_probe_copy<true>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    case 2: hipLaunchKernelGGL(k_probe_rmw<false>, dim3(grid), dim3(256), 0, s, static_cast<d2v *>(a), n, 1.0); break;
    case 3: hipLaunchKernelGGL(k_probe_rmw<true>, dim3(grid), dim3(256), 0, s, static_cast<d2v *>(a), n, 1.0); break;
    default: return -1;
  }
  return 0;
}
