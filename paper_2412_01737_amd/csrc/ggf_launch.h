// Host-side launch wrappers shared by the kernel translation units and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ggf_device.h"

// Device pointers and scalars every launch needs.
struct LaunchCtx {
  hipStream_t stream;
  int precision;                 // 64 or 32
  const ChainDev *chains;
  const TensorDev *tensors;
  void *G;                       // double* or float*
  void *F;                       // factor arena, same type as G
  int8_t *links;
  double *logw;
  double2 *sfac;
  uint32_t *sweep;
  uint32_t *acc_since;
  unsigned long long *acc_total;
  unsigned long long *prop_total;
  unsigned long long *refreshes;
  double *max_drift;
  double *ldet;
  int *flags;
  int *acc_list;                 // compacted accepted chains of the current link step
  int *acc_cnt;                  // [2] double-buffered accepted counts
  double *scratch;               // float64 refactorisation scratch
  // delayed updates (dld > 0): pending factors of the current window of link
  // steps, G_cur = G - X Y^T, chain c's X and Y n x dld row-major at x_off[c];
  // pend[c] = 1 + the window slot of the chain's last accepted flip (0: none)
  void *X, *Y;
  const size_t *x_off;
  int *pend;
  int dld;
  uint32_t key0, key1;
  int n_chains;
};

void ggf_launch_assemble(const LaunchCtx &lc, const int *list, int count, int max_sites);
void ggf_launch_gj(const LaunchCtx &lc, const int *list, int count, int n_max, int nb, int *piv,
                   int *perm, size_t piv_stride, double *ybuf);
void ggf_launch_store(const LaunchCtx &lc, const int *list, int count, int n_max, const int *perm,
                      size_t piv_stride);
void ggf_launch_post(const LaunchCtx &lc, const int *list, int count, int is_refresh);

// One link step: ratio + decision + factors, then the streaming rank-4 update
// (or, with delayed updates, the factors of window slot t).
void ggf_launch_ratio(const LaunchCtx &lc, int ell, int parity, int kmax, int t, int n_max);
// Delayed updates: G -= X Y^T for every chain with a pending flip in the window
// (matrix-core GEMM of rank 4 * pend[c] rounded up to 16); all_list holds 0..n_chains-1
// and all_cnt[0] = n_chains.
void ggf_launch_flush(const LaunchCtx &lc, const int *all_list, int *all_cnt, int grid, int n_max);
void ggf_launch_update(const LaunchCtx &lc, int parity, int grid, int tiles, int nt);
void ggf_launch_end_sweep(const LaunchCtx &lc);
void ggf_launch_hot_start(const LaunchCtx &lc, int max_links);
void ggf_launch_sfac(const LaunchCtx &lc, const int *list, int count, int kmax);
void ggf_launch_measure(const LaunchCtx &lc, uint32_t mask, double *out, int kmax);
int ggf_launch_probe(int mode, void *a, void *b, size_t bytes, int grid, hipStream_t s);
