// Stream probes: a plain copy and an in-place read-modify-write of a large
// buffer, with and without non-temporal hints, and unrolled variants (copy,
// read-modify-write, read only, write only) with 8 loads in flight per thread.
// They calibrate the HBM traffic counters and give the achievable bandwidth the
// update kernels are compared with.
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

// Unrolled probes: every wave instruction moves 1 KB of consecutive bytes and each thread keeps
// U loads in flight before its first store; a workgroup streams one contiguous chunk of the buffer.
// Modes: copy, in-place read-modify-write, read only (a sum kept per thread, stored once so that the
// loads are not dead) and write only.
constexpr int kU = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_probe_unrolled(const d2v *src, d2v *dst, size_t n) {
  const size_t per_wg = (n + gridDim.x - 1) / gridDim.x;
  const size_t lo = static_cast<size_t>(blockIdx.x) * per_wg;
  const size_t hi = lo + per_wg < n ? lo + per_wg : n;
  d2v acc = {0.0, 0.0};
  for (size_t base = lo; base < hi; base += static_cast<size_t>(kU) * blockDim.x) {
    d2v v[kU];
    if (MODE != 3) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const size_t i = base + static_cast<size_t>(u) * blockDim.x + threadIdx.x;
        v[u] = i < hi ? __builtin_nontemporal_load(src + i) : d2v{0.0, 0.0};
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const size_t i = base + static_cast<size_t>(u) * blockDim.x + threadIdx.x;
      if (i >= hi) continue;
      if (MODE == 0) __builtin_nontemporal_store(v[u], dst + i);
      else if (MODE == 1) { d2v w = v[u]; w.x = fma(w.x, 1.0, 1.0); w.y = fma(w.y, 1.0, 1.0); __builtin_nontemporal_store(w, dst + i); }
      else if (MODE == 2) acc += v[u];
      else __builtin_nontemporal_store(d2v{1.0, 2.0}, dst + i);
    }
  }
  if (MODE == 2 && acc.x == -1.0 && acc.y == -1.0) dst[0] = acc;   // never true for the probe's data
}

}  // namespace

int ggf_launch_probe(int mode, void *a, void *b, size_t bytes, int grid, hipStream_t s) {
  const size_t n = bytes / sizeof(double2);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe_copy<false>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    case 1: hipLaunchKernelGGL(k_probe_copy<true>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    case 2: hipLaunchKernelGGL(k_probe_rmw<false>, dim3(grid), dim3(256), 0, s, static_cast<d2v *>(a), n, 1.0); break;
    case 3: hipLaunchKernelGGL(k_probe_rmw<true>, dim3(grid), dim3(256), 0, s, static_cast<d2v *>(a), n, 1.0); break;
    case 4: hipLaunchKernelGGL(k_probe_unrolled<0>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    case 5: hipLaunchKernelGGL(k_probe_unrolled<1>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(a), n); break;
    case 6: hipLaunchKernelGGL(k_probe_unrolled<2>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    case 7: hipLaunchKernelGGL(k_probe_unrolled<3>, dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(a), static_cast<d2v *>(b), n); break;
    default: return -1;
  }
  return 0;
}
