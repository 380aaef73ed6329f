// Refactorisation kernels: assemble M(G) and invert it in float64 by blocked
// Gauss-Jordan elimination with partial pivoting.
//
// M(G) = D + O(G) Gamma_B0 O(G)^T is the virtual matrix whose Pfaffian gives
// the weight (Sec. 3.2 PEPS norm, Sec. 5 gauged tensor O^T Gamma_A O moved to
// the bonds): per site the 8x8 virtual block d, per link the 2x2 out-in block
// R(theta_link) x0 and its negative transpose.  log W = (1/2) log|det M| - 4V ln 2.
//
// Gauss-Jordan in column blocks of width nb.  Each block panel is factored
// recursively: its left half, the left half's transform applied to the right
// half, the right half, the right half's transform applied to the left half,
// down to base panels of 8 columns held in registers (pivot rows recorded, each
// eliminated column replaced by the corresponding column of the partial
// inverse).  A panel's transform on any other columns is its row swaps
// followed by  x <- (x with the pivot rows zeroed) + Z x[pivot rows],  Z the
// panel columns -- a rank-w update done as a register-blocked float64 GEMM.
// The final column un-permutation is folded into the store of G.
#include <algorithm>

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

// Base panel of the recursive factorisation: unblocked Gauss-Jordan on at most
// BW columns [j, j+w) of one chain, the panel held in registers (thread t owns
// rows t, t + T, ..., at most RPT of them).  Per column: block argmax of |A[r][k]|
// over rows r >= k (wave shuffles, then LDS), swap of rows k and p through LDS,
// scaling of the pivot row (its pivot entry replaced by 1/pv), elimination of the
// other rows (their entry in column k replaced by -f/pv).
template <int RPT, int BW>
__global__ __launch_bounds__(1024) void k_gj_base(const int *__restrict__ list, int count,
                                                  const ChainDev *__restrict__ chains, double *__restrict__ scr,
                                                  int *__restrict__ piv, size_t piv_stride, double *__restrict__ ldet,
                                                  int *__restrict__ flags, int j, int w) {
  const int b = blockIdx.x;
  if (b >= count) return;
  const int c = list[b];
  const ChainDev ch = chains[c];
  const int n = ch.n;
  if (j >= n) return;
  const int we = min(w, n - j);
  const int T = blockDim.x;
  double *A = scr + ch.scr_off;
  int *pv_rows = piv + static_cast<size_t>(b) * piv_stride;
  __shared__ double s_rk[BW], s_rp[BW], s_bv[16];
  __shared__ int s_bi[16];
  __shared__ int s_p;
  __shared__ double s_pv;
  double v[RPT][BW];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = threadIdx.x + q * T;
#pragma unroll
    for (int t = 0; t < BW; ++t) v[q][t] = (r < n && t < we) ? A[static_cast<size_t>(r) * n + j + t] : 0.0;
  }
  double acc_ldet = (j == 0) ? 0.0 : ldet[c];
  bool singular = false;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = T >> 6;
#pragma unroll
  for (int kk = 0; kk < BW; ++kk) {
    if (kk >= we) break;
    const int k = j + kk;
    double best = -1.0;
    int bi = n;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = threadIdx.x + q * T;
      const double a = fabs(v[q][kk]);
      if (r >= k && r < n && (a > best || (a == best && r < bi))) { best = a; bi = r; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { s_bv[wv] = best; s_bi[wv] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bb = s_bv[0];
      int ii = s_bi[0];
      for (int q = 1; q < nw; ++q)
        if (s_bv[q] > bb || (s_bv[q] == bb && s_bi[q] < ii)) { bb = s_bv[q]; ii = s_bi[q]; }
      s_p = (ii < n && bb > 0.0) ? ii : k;    // no finite nonzero pivot: keep order, flag below
      pv_rows[k] = s_p;
    }
    __syncthreads();
    const int p = s_p;
    if (p != k) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = threadIdx.x + q * T;
        if (r == k)
          for (int t = 0; t < BW; ++t) s_rk[t] = v[q][t];
        if (r == p)
          for (int t = 0; t < BW; ++t) s_rp[t] = v[q][t];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = threadIdx.x + q * T;
        if (r == k)
          for (int t = 0; t < BW; ++t) v[q][t] = s_rp[t];
        if (r == p)
          for (int t = 0; t < BW; ++t) v[q][t] = s_rk[t];
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (threadIdx.x + q * T == k) s_pv = v[q][kk];
    __syncthreads();
    const double pv = s_pv;
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) {
      singular = true;
      __syncthreads();
      continue;
    }
    acc_ldet += log(fabs(pv));
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (threadIdx.x + q * T == k) {
#pragma unroll
        for (int t = 0; t < BW; ++t) {
          v[q][t] = (t == kk ? 1.0 : v[q][t]) / pv;
          s_rk[t] = v[q][t];
        }
      }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = threadIdx.x + q * T;
      if (r == k || r >= n) continue;
      const double f = v[q][kk];
#pragma unroll
      for (int t = 0; t < BW; ++t) v[q][t] = (t == kk ? 0.0 : v[q][t]) - f * s_rk[t];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = threadIdx.x + q * T;
    if (r < n)
#pragma unroll
      for (int t = 0; t < BW; ++t)
        if (t < we) A[static_cast<size_t>(r) * n + j + t] = v[q][t];
  }
  if (threadIdx.x == 0) {
    ldet[c] = acc_ldet;
    if (singular) flags[c] |= GGF_FLAG_SINGULAR;
  }
}

// Apply the panel's row swaps to every column outside the panel (each column
// independently, swaps in order) and snapshot the nb pivot rows into Y, so the
// update can overwrite them while other tiles still read them.
__global__ __launch_bounds__(256) void k_gj_swapcopy(const int *__restrict__ list, int count,
                                                     const ChainDev *__restrict__ chains, double *__restrict__ scr,
                                                     const int *__restrict__ piv, size_t piv_stride,
                                                     double *__restrict__ ybuf, int pj, int pw, int c_lo, int c_hi) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const ChainDev ch = chains[list[b]];
  const int n = ch.n;
  if (pj >= n) return;
  const int col = c_lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= min(c_hi, n)) return;
  const int pwe = min(pw, n - pj);
  if (col >= pj && col < pj + pwe) return;     // the panel's own columns
  double *A = scr + ch.scr_off;
  const int *pr = piv + static_cast<size_t>(b) * piv_stride;
  double *Y = ybuf + ch.y_off;
  for (int t = 0; t < pwe; ++t) {
    const int r2 = pr[pj + t];
    if (r2 != pj + t) {
      double *x1 = A + static_cast<size_t>(pj + t) * n + col;
      double *x2 = A + static_cast<size_t>(r2) * n + col;
      const double tmp = *x1;
      *x1 = *x2;
      *x2 = tmp;
    }
  }
  for (int t = 0; t < pwe; ++t) Y[static_cast<size_t>(t) * n + col] = A[static_cast<size_t>(pj + t) * n + col];
}

// Rank-w update X <- (X with the pivot rows zeroed) + Z Y on columns [c_lo, c_hi)
// outside the panel, on the float64 matrix cores: a workgroup owns a 128 x 128
// tile, wave (wr, wc) its 64 x 64 quarter as 4 x 4 blocks of 16 x 16; K is
// staged through LDS in chunks of 16 with the next chunk's global loads in
// flight during the current chunk's products, and X is added in the epilogue
// (two workgroups per CU overlap one's epilogue with the other's products).
// In a 16x16x4 float64 instruction lane (li, g) = (lane % 16, lane / 16) gives
// Z[row li][k g] and Y[k g][col li] and holds X[rows g + 4 e][col li], so the
// accumulator loads and stores cover 128 contiguous bytes of a row per 16 lanes.
// Z = the panel columns (final), Y = the snapshot of the pivot rows.
// TC = columns per workgroup tile (32, 64 or 128): narrow tiles for the updates
// inside a panel, whose width is the panel half being applied.
constexpr int kGT = 128, kGK = 16;
typedef double gj_acc_t __attribute__((ext_vector_type(4)));
template <int TC>
__global__ __launch_bounds__(256, 2) void k_gj_gemm(const int *__restrict__ list, int count,
                                                 const ChainDev *__restrict__ chains, double *__restrict__ scr,
                                                 const double *__restrict__ ybuf, int pj, int pw, int c_lo, int c_hi) {
  const int b = blockIdx.z;
  if (b >= count) return;
  const ChainDev ch = chains[list[b]];
  const int n = ch.n;
  if (pj >= n) return;
  const int hi = min(c_hi, n);
  constexpr int CB = TC / 32;                          // 16-column blocks per wave
  const int r0 = blockIdx.y * kGT, c0 = c_lo + blockIdx.x * TC;
  if (r0 >= n || c0 >= hi) return;
  const int pwe = min(pw, n - pj);
  if (c0 >= pj && c0 + TC <= pj + pwe) return;      // tile entirely inside the panel
  double *A = scr + ch.scr_off;
  const double *Y = ybuf + ch.y_off;
  __shared__ double sZ[kGK][kGT + 1];
  __shared__ double sY[kGK][TC + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int wr = 64 * (w >> 1), wc = (TC / 2) * (w & 1);
  gj_acc_t acc[4][CB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[a][c] = static_cast<gj_acc_t>(0.0);
  // staging map: Z chunk by (row q = t/2, k half kh = 8 (t&1)), Y chunk by (k = t/128, col)
  const int zq = threadIdx.x >> 1, zk = (threadIdx.x & 1) * 8;
  double zreg[8], yreg[TC / 16];
  auto load_chunk = [&](int k0) {
    const int rr = r0 + zq;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int kk = zk + i;
      zreg[i] = (k0 + kk < pwe && rr < n) ? A[static_cast<size_t>(rr) * n + pj + k0 + kk] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < TC / 16; ++i) {
      const int t = threadIdx.x + 256 * i;
      const int kk = t / TC, q = t - kk * TC;
      const int cc = c0 + q;
      yreg[i] = (k0 + kk < pwe && cc < hi) ? Y[static_cast<size_t>(k0 + kk) * n + cc] : 0.0;
    }
  };
  load_chunk(0);
  for (int k0 = 0; k0 < pwe; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < 8; ++i) sZ[zk + i][zq] = zreg[i];
#pragma unroll
    for (int i = 0; i < TC / 16; ++i) {
      const int t = threadIdx.x + 256 * i;
      sY[t / TC][t % TC] = yreg[i];
    }
    __syncthreads();
    if (k0 + kGK < pwe) load_chunk(k0 + kGK);
#pragma unroll
    for (int k4 = 0; k4 < kGK; k4 += 4) {
      double zo[4], yo[CB];
#pragma unroll
      for (int a = 0; a < 4; ++a) zo[a] = sZ[k4 + g][wr + 16 * a + li];
#pragma unroll
      for (int c = 0; c < CB; ++c) yo[c] = sY[k4 + g][wc + 16 * c + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(zo[a], yo[c], acc[a][c], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: X (zero on the pivot rows) + Z Y, columns of the panel untouched; per 16-row
  // block all loads are issued before the stores (each element is read and written by its own
  // lane only, but the compiler cannot tell the stores from the next loads)
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double xv[CB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + wr + 16 * a + g + 4 * e, col = c0 + wc + 16 * c + li;
        const bool upd = r < n && col < hi && !(col >= pj && col < pj + pwe) && !(r >= pj && r < pj + pwe);
        xv[c][e] = upd ? A[static_cast<size_t>(r) * n + col] : 0.0;
      }
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + wr + 16 * a + g + 4 * e, col = c0 + wc + 16 * c + li;
        if (r < n && col < hi && !(col >= pj && col < pj + pwe))
          A[static_cast<size_t>(r) * n + col] = xv[c][e] + acc[a][c][e];
      }
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

namespace {

struct GJRun {
  const LaunchCtx &lc;
  const int *list;
  int count, n_max;
  int *piv;
  size_t piv_stride;
  double *ybuf;
};

// Apply the transform of panel [pj, pj+pw) (its row swaps, then the rank-pw update) to columns [c_lo, c_hi).
void gj_apply(const GJRun &g, int pj, int pw, int c_lo, int c_hi) {
  const int width = c_hi - c_lo;
  hipLaunchKernelGGL(k_gj_swapcopy, dim3((width + 255) / 256, g.count), dim3(256), 0, g.lc.stream, g.list, g.count,
                     g.lc.chains, g.lc.scratch, g.piv, g.piv_stride, g.ybuf, pj, pw, c_lo, c_hi);
  const dim3 rows(1, (g.n_max + kGT - 1) / kGT, g.count);
  if (width <= 32)
    hipLaunchKernelGGL(k_gj_gemm<32>, dim3((width + 31) / 32, rows.y, rows.z), dim3(256), 0, g.lc.stream, g.list,
                       g.count, g.lc.chains, g.lc.scratch, g.ybuf, pj, pw, c_lo, c_hi);
  else if (width <= 64)
    hipLaunchKernelGGL(k_gj_gemm<64>, dim3((width + 63) / 64, rows.y, rows.z), dim3(256), 0, g.lc.stream, g.list,
                       g.count, g.lc.chains, g.lc.scratch, g.ybuf, pj, pw, c_lo, c_hi);
  else
    hipLaunchKernelGGL(k_gj_gemm<128>, dim3((width + 127) / 128, rows.y, rows.z), dim3(256), 0, g.lc.stream,
                       g.list, g.count, g.lc.chains, g.lc.scratch, g.ybuf, pj, pw, c_lo, c_hi);
}

// Factor the panel columns [j, j+w): recursively, left half, its transform on the right half,
// right half, its transform on the left half; base panels of 8 columns held in registers.
void gj_panel(const GJRun &g, int j, int w) {
  // base panels in registers: <= 4 rows x 8 columns per thread up to n = 4096, 8 x 4 above;
  // the fewest threads that cover the rows (each pivot search is a workgroup reduction)
  const int T = g.n_max <= 1024 ? 256 : (g.n_max <= 2048 ? 512 : 1024);
  const int bw = g.n_max <= 4096 ? 8 : 4;
  if (w <= bw) {
    if (g.n_max <= 4096)
      hipLaunchKernelGGL((k_gj_base<4, 8>), dim3(g.count), dim3(T), 0, g.lc.stream, g.list, g.count, g.lc.chains,
                         g.lc.scratch, g.piv, g.piv_stride, g.lc.ldet, g.lc.flags, j, w);
    else
      hipLaunchKernelGGL((k_gj_base<8, 4>), dim3(g.count), dim3(T), 0, g.lc.stream, g.list, g.count, g.lc.chains,
                         g.lc.scratch, g.piv, g.piv_stride, g.lc.ldet, g.lc.flags, j, w);
    return;
  }
  const int h = w / 2;
  gj_panel(g, j, h);
  gj_apply(g, j, h, j + h, j + w);
  gj_panel(g, j + h, w - h);
  gj_apply(g, j + h, w - h, j, j + h);
}

}  // namespace

void ggf_launch_gj(const LaunchCtx &lc, const int *list, int count, int n_max, int nb, int *piv,
                   int *perm, size_t piv_stride, double *ybuf) {
  const GJRun g{lc, list, count, n_max, piv, piv_stride, ybuf};
  for (int j = 0; j < n_max; j += nb) {
    const int w = std::min(nb, n_max - j);
    gj_panel(g, j, w);
    gj_apply(g, j, w, 0, n_max);
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
