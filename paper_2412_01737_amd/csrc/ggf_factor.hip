// Refactorisation kernels: assemble M(G) and invert it in float64 by blocked
// Gauss-Jordan elimination with partial pivoting.
//
// M(G) = D + O(G) Gamma_B0 O(G)^T is the virtual matrix whose Pfaffian gives
// the weight (Sec. 3.2 PEPS norm, Sec. 5 gauged tensor O^T Gamma_A O moved to
// the bonds): per site the 8x8 virtual block d, per link the 2x2 out-in block
// R(theta_link) x0 and its negative transpose.  log W = (1/2) log|det M| - 4V ln 2.
//
// Gauss-Jordan, panel width nb: the panel kernel runs the unblocked in-place
// elimination on the n x nb panel (pivot rows recorded, the eliminated column
// replaced by the corresponding column of the partial inverse); the update
// kernel applies the panel's row swaps to every other column, then
//   x <- (x with the nb pivot rows zeroed) + Z x[pivot rows],
// Z the n x nb panel -- a rank-nb update, so all work is GEMM-shaped.  The
// final column un-permutation is folded into the store of G.
#include "ggf_device.h"
#include "ggf_launch.h"

namespace {

__global__ __launch_bounds__(256) void k_assemble(const int *__restrict__ list, int count,
                                                  const ChainDev *__restrict__ chains,
                                                  const TensorDev *__restrict__ tensors,
                                                  const int8_t *__restrict__ links,
                                                  double *__restrict__ scr) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const ChainDev ch = chains[list[b]];
  const int n = ch.n, L = ch.L;
  const int site = blockIdx.x;
  if (8 * site >= n) return;
  const TensorDev &T = tensors[ch.tensor];
  const int8_t *lk = links + ch.link_off;
  double *M = scr + ch.scr_off;
  for (int r = 0; r < 8; ++r) {
    const int i = 8 * site + r;
    const int leg = r >> 1, t = r & 1;
    // bond partner of this row: (partner site, partner leg, 2-vector of values)
    int psite, pleg;
    double v0, v1;
    double y[4];
    if (leg == 2 || leg == 1) {                     // r or u: out end of link 2*site + mu
      const int mu = (leg == 2) ? 0 : 1;
      const int ell = 2 * site + mu;
      psite = mu == 0 ? ggf_shift(site, L, 1, 0) : ggf_shift(site, L, 0, 1);
      pleg = mu == 0 ? 0 : 3;
      ggf_bond_block(T.x0, lk[ell], T.group, y);
      v0 = y[t * 2 + 0];                            // M[out_t][in_0]
      v1 = y[t * 2 + 1];                            // M[out_t][in_1]
    } else {                                        // l or d: in end of a link from the neighbour
      const int mu = (leg == 0) ? 0 : 1;
      const int src = mu == 0 ? ggf_shift(site, L, -1, 0) : ggf_shift(site, L, 0, -1);
      const int ell = 2 * src + mu;
      psite = src;
      pleg = mu == 0 ? 2 : 1;
      ggf_bond_block(T.x0, lk[ell], T.group, y);
      v0 = -y[0 * 2 + t];                           // M[in_t][out_0] = -Y[0][t]
      v1 = -y[1 * 2 + t];
    }
    const int pc0 = 8 * psite + 2 * pleg;
    double *row = M + static_cast<size_t>(i) * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double v = 0.0;
      if ((j >> 3) == site) v = T.d[r * 8 + (j & 7)];
      if (j == pc0) v += v0;
      if (j == pc0 + 1) v += v1;
      row[j] = v;
    }
  }
}

// Unblocked Gauss-Jordan on the panel columns [j, j+nbe) of one chain per workgroup.
__global__ __launch_bounds__(256) void k_gj_panel(const int *__restrict__ list, int count,
                                                  const ChainDev *__restrict__ chains,
                                                  double *__restrict__ scr, int *__restrict__ piv,
                                                  size_t piv_stride, double *__restrict__ ldet,
                                                  int *__restrict__ flags, int j, int nb) {
  const int b = blockIdx.x;
  if (b >= count) return;
  const int c = list[b];
  const ChainDev ch = chains[c];
  const int n = ch.n;
  if (j >= n) return;
  const int nbe = min(nb, n - j);
  double *A = scr + ch.scr_off;
  int *pv_rows = piv + static_cast<size_t>(b) * piv_stride;
  __shared__ double s_best[256];
  __shared__ int s_idx[256];
  __shared__ double s_rowk[64];
  __shared__ double s_pv;
  __shared__ int s_p;
  double acc_ldet = (j == 0) ? 0.0 : ldet[c];
  bool singular = false;
  for (int kk = 0; kk < nbe; ++kk) {
    const int k = j + kk;
    // pivot search over rows >= k in column k
    double best = -1.0;
    int bi = n;
    for (int r = k + threadIdx.x; r < n; r += blockDim.x) {
      const double v = fabs(A[static_cast<size_t>(r) * n + k]);
      if (v > best) { best = v; bi = r; }
    }
    s_best[threadIdx.x] = best;
    s_idx[threadIdx.x] = bi;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        const double ob = s_best[threadIdx.x + off];
        const int oi = s_idx[threadIdx.x + off];
        if (ob > s_best[threadIdx.x] || (ob == s_best[threadIdx.x] && oi < s_idx[threadIdx.x])) {
          s_best[threadIdx.x] = ob;
          s_idx[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    // no finite nonzero candidate: keep the row order (in-range pivot), flag singular
    const int p = (s_idx[0] < n && s_best[0] > 0.0) ? s_idx[0] : k;
    if (threadIdx.x == 0) pv_rows[k] = p;
    if (p != k && threadIdx.x < nbe) {
      double *rk = A + static_cast<size_t>(k) * n + j;
      double *rp = A + static_cast<size_t>(p) * n + j;
      const double t = rk[threadIdx.x];
      rk[threadIdx.x] = rp[threadIdx.x];
      rp[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_pv = A[static_cast<size_t>(k) * n + k];
    __syncthreads();
    const double pv = s_pv;
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) {   // singular column: skip it, indices stay valid
      singular = true;
      __syncthreads();
      continue;
    }
    acc_ldet += log(fabs(pv));
    if (threadIdx.x < nbe) {
      double *rk = A + static_cast<size_t>(k) * n + j;
      const double v = (threadIdx.x == kk) ? 1.0 / pv : rk[threadIdx.x] / pv;
      rk[threadIdx.x] = v;
      s_rowk[threadIdx.x] = v;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      if (r == k) continue;
      double *ar = A + static_cast<size_t>(r) * n + j;
      const double f = ar[kk];
      if (f == 0.0) continue;
      for (int t = 0; t < nbe; ++t) {
        const double old = (t == kk) ? 0.0 : ar[t];
        ar[t] = old - f * s_rowk[t];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ldet[c] = acc_ldet;
    if (singular) flags[c] |= GGF_FLAG_SINGULAR;
  }
}

// Rank-nb update of all columns outside the panel, 64 columns per workgroup.
template <int NB>
__global__ __launch_bounds__(256) void k_gj_update(const int *__restrict__ list, int count,
                                                   const ChainDev *__restrict__ chains,
                                                   double *__restrict__ scr,
                                                   const int *__restrict__ piv, size_t piv_stride,
                                                   int j, int nb) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const ChainDev ch = chains[list[b]];
  const int n = ch.n;
  if (j >= n) return;
  const int c0 = blockIdx.x * 64;
  if (c0 >= n) return;
  const int nbe = min(nb, n - j);
  double *A = scr + ch.scr_off;
  const int *pr = piv + static_cast<size_t>(b) * piv_stride;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = c0 + lane;
  const bool active = col < n && !(col >= j && col < j + nbe);
  if (wave == 0 && active) {
    for (int t = 0; t < nbe; ++t) {
      const int r2 = pr[j + t];
      if (r2 != j + t) {
        double *x1 = A + static_cast<size_t>(j + t) * n + col;
        double *x2 = A + static_cast<size_t>(r2) * n + col;
        const double tmp = *x1;
        *x1 = *x2;
        *x2 = tmp;
      }
    }
  }
  __syncthreads();
  double y[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) y[t] = (active && t < nbe) ? A[static_cast<size_t>(j + t) * n + col] : 0.0;
  __syncthreads();
  if (!active) return;
  for (int r = wave; r < n; r += 4) {
    const double *z = A + static_cast<size_t>(r) * n + j;   // panel row r (uniform per wave)
    double x = (r >= j && r < j + nbe) ? 0.0 : A[static_cast<size_t>(r) * n + col];
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < nbe) x = fma(z[t], y[t], x);
    A[static_cast<size_t>(r) * n + col] = x;
  }
}

// Column permutation that undoes the row pivoting: result column q = panel-ordered column arr[q].
__global__ void k_gj_perm(const int *__restrict__ list, int count, const ChainDev *__restrict__ chains,
                          const int *__restrict__ piv, size_t piv_stride, int *__restrict__ perm) {
  const int b = blockIdx.x;
  if (b >= count || threadIdx.x != 0) return;
  const int n = chains[list[b]].n;
  const int *pr = piv + static_cast<size_t>(b) * piv_stride;
  int *arr = perm + static_cast<size_t>(b) * piv_stride;
  for (int q = 0; q < n; ++q) arr[q] = q;
  for (int k = n - 1; k >= 0; --k) {
    const int p = pr[k];
    const int t = arr[k];
    arr[k] = arr[p];
    arr[p] = t;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gj_store(const int *__restrict__ list, int count,
                                                  const ChainDev *__restrict__ chains,
                                                  const double *__restrict__ scr,
                                                  const int *__restrict__ perm, size_t piv_stride,
                                                  T *__restrict__ G) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const ChainDev ch = chains[list[b]];
  const int n = ch.n;
  const int r0 = blockIdx.x * 8;
  if (r0 >= n) return;
  const double *A = scr + ch.scr_off;
  const int *arr = perm + static_cast<size_t>(b) * piv_stride;
  T *out = G + ch.g_off;
  for (int r = r0; r < min(r0 + 8, n); ++r)
    for (int q = threadIdx.x; q < n; q += blockDim.x)
      out[static_cast<size_t>(r) * n + q] = static_cast<T>(A[static_cast<size_t>(r) * n + arr[q]]);
}

// log W from log|det M|; drift bookkeeping on refreshes.
__global__ void k_gj_post(const int *__restrict__ list, int count, const ChainDev *__restrict__ chains,
                          const double *__restrict__ ldet, double *__restrict__ logw,
                          double *__restrict__ max_drift, uint32_t *__restrict__ acc_since,
                          unsigned long long *__restrict__ refreshes, int is_refresh) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  const int c = list[b];
  const int V = chains[c].L * chains[c].L;
  const double lw = 0.5 * ldet[c] - 4.0 * V * 0.69314718055994530942;
  if (is_refresh) {
    const double d = fabs(lw - logw[c]);
    if (!(d <= max_drift[c])) max_drift[c] = d;
    refreshes[c] += 1;
  }
  logw[c] = lw;
  acc_since[c] = 0;
}

}  // namespace

void ggf_launch_assemble(const LaunchCtx &lc, const int *list, int count, int max_sites) {
  dim3 grid(max_sites, count);
  hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, lc.stream, list, count, lc.chains, lc.tensors,
                     lc.links, lc.scratch);
}

void ggf_launch_gj(const LaunchCtx &lc, const int *list, int count, int n_max, int nb, int *piv,
                   int *perm, size_t piv_stride) {
  for (int j = 0; j < n_max; j += nb) {
    hipLaunchKernelGGL(k_gj_panel, dim3(count), dim3(256), 0, lc.stream, list, count, lc.chains,
                       lc.scratch, piv, piv_stride, lc.ldet, lc.flags, j, nb);
    dim3 grid((n_max + 63) / 64, count);
    if (nb <= 16)
      hipLaunchKernelGGL(k_gj_update<16>, grid, dim3(256), 0, lc.stream, list, count, lc.chains,
                         lc.scratch, piv, piv_stride, j, nb);
    else if (nb <= 32)
      hipLaunchKernelGGL(k_gj_update<32>, grid, dim3(256), 0, lc.stream, list, count, lc.chains,
                         lc.scratch, piv, piv_stride, j, nb);
    else
      hipLaunchKernelGGL(k_gj_update<64>, grid, dim3(256), 0, lc.stream, list, count, lc.chains,
                         lc.scratch, piv, piv_stride, j, nb);
  }
  hipLaunchKernelGGL(k_gj_perm, dim3(count), dim3(64), 0, lc.stream, list, count, lc.chains, piv,
                     piv_stride, perm);
}

void ggf_launch_store(const LaunchCtx &lc, const int *list, int count, int n_max, const int *perm,
                      size_t piv_stride) {
  dim3 grid((n_max + 7) / 8, count);
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_gj_store<double>, grid, dim3(256), 0, lc.stream, list, count, lc.chains,
                       lc.scratch, perm, piv_stride, static_cast<double *>(lc.G));
  else
    hipLaunchKernelGGL(k_gj_store<float>, grid, dim3(256), 0, lc.stream, list, count, lc.chains,
                       lc.scratch, perm, piv_stride, static_cast<float *>(lc.G));
}

void ggf_launch_post(const LaunchCtx &lc, const int *list, int count, int is_refresh) {
  hipLaunchKernelGGL(k_gj_post, dim3((count + 255) / 256), dim3(256), 0, lc.stream, list, count,
                     lc.chains, lc.ldet, lc.logw, lc.max_drift, lc.acc_since, lc.refreshes, is_refresh);
}
