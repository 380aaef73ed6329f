// Sweep and measurement kernels: the single-link Metropolis step (Sec. 5.1
// sampling of p(G) = N(G)/N) on the maintained inverse G = M(G)^-1.
//
// Link step l, per chain (k_ratio, one workgroup per chain):
//   U = (out0, out1, in0, in1) Majoranas of link l; the proposal changes the
//   out-in block of M by X = (R(theta') - R(theta)) x0, i.e. dM_UU = [[0, X], [-X^T, 0]];
//   rho = det(1 + G_UU dM_UU) = (W'/W)^2 by the matrix determinant lemma;
//   for K > 1, S' = N(G')/W(G') from the patch Pfaffians of every pair (n, m)
//   of the superposition evaluated on G' restricted to the patch Majoranas
//   (Woodbury: G'_SS = G_SS + G_SU K G_SU^T);
//   accept iff u < sqrt(rho) S'/S with u from Philox(chain, sweep, link, 0).
//   On accept the workgroup writes PT = -G[U,:] and QT = (G[:,U] K)^T,
//   K = dM (1 + G_UU dM)^-1 = (dM^-1 + G_UU)^-1, and appends the chain to the
//   step's accepted list.
// Then the streaming update (k_update) applies G <- G + QT^T PT
// = G - G[:,U] K G[U,:] to every accepted chain, each element once: read n^2, write n^2.
//
// Delayed updates (lc.dly = F > 0): the flips of a window of F link steps are
// not applied at once.  With A the Majoranas of the flips accepted so far in the
// window and dM_A their block-diagonal change, the current inverse is
//   G_cur = G - G[:,A] W G[A,:],  W = dM_A Binv,  Binv = (1 + G_AA dM_A)^-1
// (block Woodbury; the same chain as one update per flip).  A link step only
// needs G_cur on the link's and the patch links' Majoranas I, i.e. G_II, G_IA
// and G_AI gathered from the unchanged G; an accepted flip borders Binv by its 4
// rows and columns (Schur complement S = 1 + G_cur,UU dM, whose determinant is
// rho).  At the end of the window the block-update kernels apply the whole
// window as one rank-|A| matrix-core update of G.
#include <mutex>
#include <type_traits>

#include "ggf_device.h"
#include "ggf_launch.h"
#include "ggf_nn.h"
#include "ggf_pair.h"

namespace {

constexpr int kDelayMax = GGF_BLOCK_RMAX;   // Majoranas pending in a window (4 per flip; the block-update rank limit)

constexpr int kRatioThreads = 64;   // one wave per chain: the per-step work is small, residency is what counts

// PAIRS: some chain of the context has K > 1 (patch Pfaffians; index sets up to 16 Majoranas).
template <typename T, bool PAIRS>
__global__ __launch_bounds__(kRatioThreads) void k_ratio(LaunchCtx lc, int step, int parity, int t, int wp) {
  extern __shared__ double2 s_work[];   // pair workspaces, then (delayed) G_IA, G_AI and a scratch block
  __shared__ double s_K[16], s_Ai[16], s_dM[16], s_Am[16];
  __shared__ double s_GI[(PAIRS ? 16 : 4) * 16];   // current inverse on the Majoranas I (U first), row stride 16
  __shared__ int s_I[16];
  __shared__ int s_nI;
  __shared__ double s_rho, s_u;
  __shared__ int s_kn, s_acc;
  __shared__ double2 s_r[16];
  __shared__ double2 s_tv[PAIRS ? kRatioThreads / kPairLanes : 1][32];   // pair elimination scratch
  const int c = blockIdx.x;
  const bool delayed = lc.dly > 0;
  if (c == 0 && threadIdx.x == 0) {
    if (!delayed) lc.acc_cnt[parity ^ 1] = 0;
    else if (t == 0) lc.dcnt[wp ^ 1] = 0;          // the other window's list was flushed already
  }
  const ChainDev ch = lc.chains[c];
  const int n = ch.n;
  const int a = (delayed && t > 0) ? lc.dr[c] : 0;  // pending Majoranas of this chain
  if (delayed && t == 0 && threadIdx.x == 0) lc.dr[c] = 0;
  // the link of this step: the step itself (link steps in lock-step, chains past their last link
  // idle), or with balanced sweeps the chain's own cursor (every chain steps every time and starts
  // its next sweep when it wraps)
  const int ell = lc.cursor ? lc.cursor[c] : step;
  if (ell >= ch.nlinks) return;
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  int8_t *lk = lc.links + ch.link_off;
  int U[4];
  ggf_link_u(ell, ch.L, U);
  if (!PAIRS && delayed && a + 4 <= kDelayMax) {
    // rows U of the stored G (unchanged within the window) become rows a .. a + 3 of the
    // window's P = G[A,:], read by the flush if this flip is accepted; a rejected step's
    // rows are overwritten by the next accepted one (with pairs the workgroups are fewer per
    // CU, the copy does not hide, and the flush copies the rows itself)
    typedef typename std::conditional<sizeof(T) == 8, d2v, f4v>::type V;
    constexpr int VW = 16 / sizeof(T);
    T *P = static_cast<T *>(lc.dP) + lc.dP_off[c] + static_cast<size_t>(a) * n;
    const int nv = n / VW;
#pragma unroll 8
    for (int e = threadIdx.x; e < 4 * nv; e += blockDim.x) {
      const int q = e / nv, v = e - q * nv;
      reinterpret_cast<V *>(P + static_cast<size_t>(q) * n)[v] =
          reinterpret_cast<const V *>(G + static_cast<size_t>(U[q]) * n)[v];
    }
  }
  const int K = PAIRS ? ch.K : 1;
  const int npairs = K * (K + 1) / 2 - 1;
  if (threadIdx.x == 0) {
    // index set: U first, then the Majoranas of every patch link of the superposition
    int m = 0;
    for (int q = 0; q < 4; ++q) s_I[m++] = U[q];
    for (int p = 0; p < npairs; ++p) {
      int pa, pb;
      pair_of(p, K, pa, pb);
      for (int l = 0; l < Tn.nl[pa][pb]; ++l) {
        int u4[4];
        ggf_link_u(Tn.lk[pa][pb][l], ch.L, u4);
        for (int q = 0; q < 4; ++q) {
          bool seen = false;
          for (int i = 0; i < m; ++i) seen |= s_I[i] == u4[q];
          if (!seen && m < 16) s_I[m++] = u4[q];
        }
      }
    }
    s_nI = m;
  }
  __syncthreads();
  const int nI = s_nI;
  // delayed-window work arrays after the pair workspaces, nIm the largest index set (4 Majoranas
  // when K = 1): s_H (nIm x a) = G_IA, then H = G_IA dM_A in place; s_GAI (a x nIm) = G_AI;
  // s_T ((nIm + 4) x a): T = H Binv in rows [0, nI), b12 in rows [nIm, nIm + 4)
  const int nIm = PAIRS ? lc.nidx : 4;
  const int lda = 4 * lc.dly;            // >= a + 4: pending Majoranas of a full window
  double *s_H = reinterpret_cast<double *>(s_work + (npairs > 0 ? npairs * kPairLd * kPairLd : 0));
  double *s_GAI = s_H + nIm * lda;
  double *s_T = s_GAI + nIm * lda;
  const int *A = delayed ? lc.dU + static_cast<size_t>(c) * kDelayMax : nullptr;
  const double *dXc = delayed ? lc.dX + static_cast<size_t>(c) * kDelayMax : nullptr;   // X of each pending flip
  const double *Binv = delayed ? lc.dBinv + static_cast<size_t>(c) * kDelayMax * kDelayMax : nullptr;
  if (a > 0) {
    for (int e = threadIdx.x; e < nI * a; e += blockDim.x) {
      const int i = e / a, p = e - i * a;
      s_H[i * lda + p] = static_cast<double>(G[static_cast<size_t>(s_I[i]) * n + A[p]]);
      s_GAI[p * nIm + i] = static_cast<double>(G[static_cast<size_t>(A[p]) * n + s_I[i]]);
    }
    __syncthreads();
    // H = G_IA dM_A, one 4-column block of one row per thread: dM_A is block diagonal with
    // blocks [[0, X], [-X^T, 0]], X = (X0 X1; X2 X3) of the pending flip
    for (int e = threadIdx.x; e < nI * (a / 4); e += blockDim.x) {
      const int i = e / (a / 4), blk = 4 * (e - i * (a / 4));
      double *h = s_H + i * lda + blk;
      const double *X = dXc + blk;
      const double g0 = h[0], g1 = h[1], g2 = h[2], g3 = h[3];
      h[0] = -g2 * X[0] - g3 * X[1];
      h[1] = -g2 * X[2] - g3 * X[3];
      h[2] = g0 * X[0] + g1 * X[2];
      h[3] = g0 * X[1] + g1 * X[3];
    }
    __syncthreads();
    // T = H Binv = G_IA W, W = dM_A Binv: one column q of Binv per thread, read once for all
    // rows of T, 8 loads in flight
    constexpr int kNI = PAIRS ? 16 : 4;   // register bound of the index set
    for (int q = threadIdx.x; q < a; q += blockDim.x) {
      double v[kNI];
#pragma unroll
      for (int i = 0; i < kNI; ++i) v[i] = 0.0;
      for (int p0 = 0; p0 < a; p0 += 8) {
        double bq[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          bq[k] = p0 + k < a ? Binv[static_cast<size_t>(p0 + k) * kDelayMax + q] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
          for (int i = 0; i < kNI; ++i)
            if (i < nI && p0 + k < a) v[i] += s_H[i * lda + p0 + k] * bq[k];
      }
#pragma unroll
      for (int i = 0; i < kNI; ++i)
        if (i < nI) s_T[i * lda + q] = v[i];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nI * nI; e += blockDim.x) {
    const int i = e / nI, j = e - i * nI;
    double v = static_cast<double>(G[static_cast<size_t>(s_I[i]) * n + s_I[j]]);
    for (int q = 0; q < a; ++q) v -= s_T[i * lda + q] * s_GAI[q * nIm + j];
    s_GI[i * 16 + j] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int kold = lk[ell];
    const uint4 x = ggf_philox(make_uint4(static_cast<uint32_t>(c), lc.sweep[c], static_cast<uint32_t>(ell), 0u),
                               lc.key0, lc.key1);
    // Z_N proposal: a step of 1 + (x.z mod (N - 1)), uniform over the other N - 1 elements
    const int kn = (kold + 1 + static_cast<int>(x.z % static_cast<uint32_t>(ch.group - 1))) % ch.group;
    double yo[4], yn[4];
    ggf_bond_block(Tn.x0, kold, ch.group, yo);
    ggf_bond_block(Tn.x0, kn, ch.group, yn);
    const double X0 = yn[0] - yo[0], X1 = yn[1] - yo[1], X2 = yn[2] - yo[2], X3 = yn[3] - yo[3];
    const double dM[16] = {0, 0, X0, X1, 0, 0, X2, X3, -X0, -X2, 0, 0, -X1, -X3, 0, 0};
    // the 4x4 system lives in LDS (s_Am, s_Ai): its pivoting on registers would set the
    // register budget of the whole kernel
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double v = (i == j) ? 1.0 : 0.0;
        for (int q = 0; q < 4; ++q) v += s_GI[i * 16 + q] * dM[q * 4 + j];
        s_Am[i * 4 + j] = v;
        s_Ai[i * 4 + j] = (i == j) ? 1.0 : 0.0;
      }
    const double rho = ggf_solve4(s_Am, s_Ai);      // s_Ai <- (1 + G_UU dM)^-1
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v += dM[i * 4 + q] * s_Ai[q * 4 + j];
        s_K[i * 4 + j] = v;
      }
    for (int q = 0; q < 16; ++q) s_dM[q] = dM[q];
    s_rho = rho;
    s_kn = kn;
    s_u = ggf_u53(x.x, x.y);
  }
  __syncthreads();
  if (PAIRS && K > 1) {
    // pairs 8 at a time, 8 lanes each (K = 1 .. 4: at most 9 pairs); K is uniform in the workgroup
    const int grp = threadIdx.x / kPairLanes, gl = threadIdx.x % kPairLanes;
    for (int p0 = 0; p0 < npairs; p0 += kRatioThreads / kPairLanes) {
      const int p = p0 + grp;
      const bool act = p < npairs;
      PatchSet ps;
      ps.s = 0;
      int pa = 0, pb = 0;
      double2 *Wp = s_work + (act ? p : 0) * kPairLd * kPairLd;
      if (act) {
        pair_of(p, K, pa, pb);
        pair_set(Tn, pa, pb, ch.L, ps);
        build_pair_rows(Tn, pa, pb, ch.group, s_GI, s_I, nI, lk, s_K, ell, s_kn, ps, Wp, gl);
      }
      __syncthreads();
      double2 pf = pfaffian_lanes(Wp, act ? 2 * ps.s : 0, s_tv[grp], gl);
      if (act && gl == 0) {
        if ((ps.s / 2) & 1) pf = cscale(pf, -1.0);   // r = (-1)^(s/2) Pf, as pair_ratio
        s_r[p] = pf;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const double rho = s_rho;
    double2 snew = make_double2(1.0, 0.0);
    double sratio = 1.0;
    if (PAIRS && K > 1) {
      double sv = Tn.w[0][0].x;
      for (int p = 0; p < npairs; ++p) {
        int pa, pb;
        pair_of(p, K, pa, pb);
        const double2 tt = cmul(Tn.w[pa][pb], s_r[p]);
        sv += (pa == pb) ? tt.x : 2.0 * tt.x;
      }
      snew = make_double2(sv, 0.0);
      sratio = sv / lc.sfac[c].x;
    }
    const bool bad = !isfinite(rho) || !isfinite(sratio) || rho < -1e-6;
    const double R = (rho > 0.0 ? sqrt(rho) : 0.0) * sratio;
    const bool accept = !bad && (s_u < R) && (a + 4 <= kDelayMax || !delayed);
    lc.prop_total[c] += 1;
    if (!bad && fabs(s_u - R) < 1e-9 * R) lc.ties[c] += 1;
    if (bad) lc.flags[c] |= GGF_FLAG_NONFINITE;
    if (accept) {
      lk[ell] = static_cast<int8_t>(s_kn);
      lc.logw[c] += 0.5 * log(rho);
      lc.sfac[c] = snew;
      lc.acc_since[c] += 1;
      lc.acc_total[c] += 1;
      if (delayed) {
        if (a == 0) {
          const int slot = atomicAdd(lc.dcnt + wp, 1);
          lc.acc_list[slot] = c;
        }
      } else {
        const int slot = atomicAdd(lc.acc_cnt + parity, 1);
        lc.acc_list[slot] = c;
      }
    }
    s_acc = accept ? 1 : 0;
    if (lc.cursor) {
      if (ell + 1 == ch.nlinks) {
        lc.cursor[c] = 0;
        lc.sweep[c] += 1;
      } else {
        lc.cursor[c] = ell + 1;
      }
    }
  }
  __syncthreads();
  if (!s_acc) return;
  if (delayed) {
    // border Binv (a x a, leading dimension kDelayMax) by the flip's rows and columns:
    //   B' = [[B, b12], [b21, S]],  b12 = G_AU dM,  b21 = G_UA dM_A,  S = 1 + G_cur,UU dM (S^-1 = s_Ai),
    //   B'^-1 = [[Binv + u S^-1 v, -u S^-1], [-S^-1 v, S^-1]],  u = Binv b12,  v = b21 Binv.
    // b21 = H[U rows], so v = T[U rows] (rows 0 .. 3 of T, U being first in I).
    double *BinvW = lc.dBinv + static_cast<size_t>(c) * kDelayMax * kDelayMax;
    double *dXw = lc.dX + static_cast<size_t>(c) * kDelayMax;
    int *Ac = lc.dU + static_cast<size_t>(c) * kDelayMax;
    double *b12 = s_T + nIm * lda;       // a x 4
    double *uu = s_GAI;                  // a x 4: u (G_AI is dead once b12 is formed)
    double *Sv = s_H;                    // 4 x a: S^-1 v (H is dead once T is formed)
    if (a > 0) {
      for (int e = threadIdx.x; e < 4 * a; e += blockDim.x) {
        const int p = e >> 2, y = e & 3;
        double v = 0.0;
        for (int x = 0; x < 4; ++x) v += s_GAI[p * nIm + x] * s_dM[x * 4 + y];
        b12[p * 4 + y] = v;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < a; i += blockDim.x) {
        double u4[4] = {0, 0, 0, 0};
        const double *bi = BinvW + static_cast<size_t>(i) * kDelayMax;
        for (int j = 0; j < a; ++j) {
          const double bij = bi[j];
#pragma unroll
          for (int x = 0; x < 4; ++x) u4[x] += bij * b12[j * 4 + x];
        }
#pragma unroll
        for (int y = 0; y < 4; ++y) uu[i * 4 + y] = u4[y];
      }
      for (int e = threadIdx.x; e < 4 * a; e += blockDim.x) {
        const int x = e / a, j = e - x * a;
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < 4; ++y) v += s_Ai[x * 4 + y] * s_T[y * lda + j];
        Sv[x * lda + j] = v;
      }
      __syncthreads();
    }
    const int a2 = a + 4;
    // one column j of Binv' per thread, rows in batches of 8: every element is read and written
    // by its own thread only, so a batch's loads are all issued before its stores
    for (int j = threadIdx.x; j < a2; j += blockDim.x) {
      for (int i0 = 0; i0 < a2; i0 += 8) {
        double old[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k;
          old[k] = (i < a && j < a) ? BinvW[static_cast<size_t>(i) * kDelayMax + j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k;
          if (i >= a2) break;
          double v;
          if (i < a && j < a) {
            v = old[k];
#pragma unroll
            for (int y = 0; y < 4; ++y) v += uu[i * 4 + y] * Sv[y * lda + j];
          } else if (i < a) {
            v = 0.0;   // -(u S^-1)[i][j - a]
#pragma unroll
            for (int x = 0; x < 4; ++x) v -= uu[i * 4 + x] * s_Ai[x * 4 + (j - a)];
          } else if (j < a) {
            v = -Sv[(i - a) * lda + j];
          } else {
            v = s_Ai[(i - a) * 4 + (j - a)];
          }
          BinvW[static_cast<size_t>(i) * kDelayMax + j] = v;
        }
      }
    }
    if (threadIdx.x == 0) {
      for (int q = 0; q < 4; ++q) Ac[a + q] = U[q];
      dXw[a + 0] = s_dM[2];
      dXw[a + 1] = s_dM[3];
      dXw[a + 2] = s_dM[6];
      dXw[a + 3] = s_dM[7];
      lc.dr[c] = a2;
    }
    return;
  }
  // Woodbury with the stored rows and columns: G' = G - G[:,U] K G[U,:].
  // (Substituting -G[U,:]^T for G[:,U] would assume exact antisymmetry; rounding
  // breaks it and the symmetric part of the error then grows with every flip.)
  const int u0 = U[0], u1 = U[1], u2 = U[2], u3 = U[3];
  T *PT = static_cast<T *>(lc.F) + ch.f_off;
  T *QT = PT + 4 * static_cast<size_t>(n);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const T *gj = G + static_cast<size_t>(j) * n;
    const double c0 = static_cast<double>(gj[u0]), c1 = static_cast<double>(gj[u1]);
    const double c2 = static_cast<double>(gj[u2]), c3 = static_cast<double>(gj[u3]);
    PT[j] = static_cast<T>(-static_cast<double>(G[static_cast<size_t>(u0) * n + j]));
    PT[n + j] = static_cast<T>(-static_cast<double>(G[static_cast<size_t>(u1) * n + j]));
    PT[2 * n + j] = static_cast<T>(-static_cast<double>(G[static_cast<size_t>(u2) * n + j]));
    PT[3 * n + j] = static_cast<T>(-static_cast<double>(G[static_cast<size_t>(u3) * n + j]));
#pragma unroll
    for (int b = 0; b < 4; ++b)
      QT[static_cast<size_t>(b) * n + j] =
          static_cast<T>(c0 * s_K[0 * 4 + b] + c1 * s_K[1 * 4 + b] + c2 * s_K[2 * 4 + b] + c3 * s_K[3 * 4 + b]);
  }
}

template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef d2v type; static constexpr int n = 2; };
template <> struct Vec16<float> { typedef f4v type; static constexpr int n = 4; };
// Two adjacent elements of G (8-byte aligned for float, 16-byte for double at even offsets).
template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double2 type; };
template <> struct Vec2<float> { typedef float2 type; };

template <typename V, typename S>
__device__ __forceinline__ void upd(V &g, S q0, S q1, S q2, S q3, const V &p0, const V &p1, const V &p2,
                                    const V &p3) {
  g = q0 * p0 + (q1 * p1 + (q2 * p2 + (q3 * p3 + g)));
}

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V *p) {
  if (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ void st(V *p, const V &v) {
  if (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Streaming rank-4 update G <- G + sum_b QT[b] (x) PT[b] over the step's accepted chains.
// Work item = (accepted chain, row tile); a persistent grid strides over items.
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w on XCD
// w mod 8), each with its own L2: every row tile of an accepted chain goes to
// the same XCD so the chain's factor rows PT/QT are fetched into one L2 only.
// NT: non-temporal loads/stores of G (each element is touched once per launch).
template <typename T, bool NT>
__global__ __launch_bounds__(256) void k_update(LaunchCtx lc, int parity, int tiles) {
  typedef typename Vec16<T>::type V;
  constexpr int VW = Vec16<T>::n;
  constexpr int kXcd = 8;
  const int nacc = lc.acc_cnt[parity];
  const int xcd = blockIdx.x % kXcd;
  const int nwg = gridDim.x / kXcd;                 // workgroups per XCD (grid is a multiple of 8)
  const int nslots = (nacc > xcd) ? (nacc - xcd + kXcd - 1) / kXcd : 0;   // slots xcd, xcd+8, ...
  const int total = nslots * tiles;
  for (int item = blockIdx.x / kXcd; item < total; item += nwg) {
    const int slot = (item / tiles) * kXcd + xcd;
    const int tile = item - (item / tiles) * tiles;
    const int c = lc.acc_list[slot];
    const ChainDev ch = lc.chains[c];
    const int n = ch.n;
    const int r0 = static_cast<int>((static_cast<long>(tile) * n) / tiles);
    const int r1 = static_cast<int>((static_cast<long>(tile + 1) * n) / tiles);
    T *G = static_cast<T *>(lc.G) + ch.g_off;
    const T *PT = static_cast<const T *>(lc.F) + ch.f_off;
    const T *QT = PT + 4 * static_cast<size_t>(n);
    for (int j0 = threadIdx.x * VW; j0 < n; j0 += 256 * VW) {
      const V p0 = *reinterpret_cast<const V *>(PT + j0);
      const V p1 = *reinterpret_cast<const V *>(PT + n + j0);
      const V p2 = *reinterpret_cast<const V *>(PT + 2 * n + j0);
      const V p3 = *reinterpret_cast<const V *>(PT + 3 * n + j0);
      // rows in groups of 4, the next group's G and QT loads issued before this group's stores
      int i = r0;
      V ga[4];
      T qa[4][4];
      auto fetch = [&](int i0, V (&g)[4], T (&qq)[4][4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          g[q] = ld<NT>(reinterpret_cast<const V *>(G + static_cast<size_t>(i0 + q) * n + j0));
#pragma unroll
          for (int b = 0; b < 4; ++b) qq[q][b] = QT[b * n + i0 + q];
        }
      };
      if (i + 4 <= r1) fetch(i, ga, qa);
      for (; i + 4 <= r1; i += 4) {
        V gb[4];
        T qb[4][4];
        if (i + 8 <= r1) fetch(i + 4, gb, qb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          upd(ga[q], qa[q][0], qa[q][1], qa[q][2], qa[q][3], p0, p1, p2, p3);
          st<NT>(reinterpret_cast<V *>(G + static_cast<size_t>(i + q) * n + j0), ga[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ga[q] = gb[q];
#pragma unroll
          for (int b = 0; b < 4; ++b) qa[q][b] = qb[q][b];
        }
      }
      for (; i < r1; ++i) {
        V g = ld<NT>(reinterpret_cast<const V *>(G + static_cast<size_t>(i) * n + j0));
        upd(g, QT[i], QT[n + i], QT[2 * n + i], QT[3 * n + i], p0, p1, p2, p3);
        st<NT>(reinterpret_cast<V *>(G + static_cast<size_t>(i) * n + j0), g);
      }
    }
  }
}

__global__ void k_end_sweep(LaunchCtx lc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < lc.n_chains && !lc.cursor) lc.sweep[c] += 1u;   // balanced sweeps advance it per chain
  if (c < 2) lc.acc_cnt[c] = 0;   // every sweep starts with both accepted counters cleared
  if (c < 2 && lc.dcnt) lc.dcnt[c] = 0;
}

__global__ void k_hot_start(LaunchCtx lc, int max_links) {
  const int c = blockIdx.y;
  const ChainDev ch = lc.chains[c];
  for (int ell = blockIdx.x * blockDim.x + threadIdx.x; ell < ch.nlinks; ell += gridDim.x * blockDim.x) {
    const uint4 x = ggf_philox(make_uint4(static_cast<uint32_t>(c), 0xFFFFFFFFu, static_cast<uint32_t>(ell), 1u),
                               lc.key0, lc.key1);
    lc.links[ch.link_off + ell] = static_cast<int8_t>(x.x % static_cast<uint32_t>(ch.group));
  }
}

// S(G) = sum_nm lambda_n^* lambda_m <B_m|B_n> r_nm(G) of the committed configuration.
template <typename T>
__global__ __launch_bounds__(64) void k_sfac(LaunchCtx lc, const int *list, int count) {
  extern __shared__ double2 s_work[];
  __shared__ double2 s_r[16];
  const int bi = blockIdx.x;
  if (bi >= count) return;
  const int c = list[bi];
  const ChainDev ch = lc.chains[c];
  const int K = ch.K;
  if (K == 1) {
    if (threadIdx.x == 0) lc.sfac[c] = make_double2(1.0, 0.0);
    return;
  }
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  const int npairs = K * (K + 1) / 2 - 1;
  if (threadIdx.x < npairs) {
    int a, b;
    pair_of(threadIdx.x, K, a, b);
    PatchSet ps;
    double2 *W = s_work + threadIdx.x * kPairLd * kPairLd;
    build_pair_matrix(Tn, a, b, ch.L, ch.group, plain_view(G, ch.n), lk, nullptr, nullptr, -1, 0, W, ps);
    s_r[threadIdx.x] = pair_ratio(W, ps.s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sv = Tn.w[0][0].x;
    for (int p = 0; p < npairs; ++p) {
      int a, b;
      pair_of(p, K, a, b);
      const double2 t = cmul(Tn.w[a][b], s_r[p]);
      sv += (a == b) ? t.x : 2.0 * t.x;
    }
    lc.sfac[c] = make_double2(sv, 0.0);
    if (!isfinite(sv)) lc.flags[c] |= GGF_FLAG_NONFINITE;
  }
}

__device__ inline double2 link_phase(int k, int group) {
  if (k == 0) return make_double2(1.0, 0.0);
  if (group == 2) return make_double2(-1.0, 0.0);
  double s, co;
  sincospi(2.0 * k / group, &s, &co);
  return make_double2(co, s);
}

__device__ inline double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// Observables of one chain per workgroup (Sec. 2.3, 5.1, 5.2, 5.3).  Fermionic
// two-point functions: Gamma_out = A + B M^-1 B^T (per pair (a, b) of the
// superposition with M_ab^-1 = G - G_S Y_ab G_S^T, Y_ab = Delta (1 + G_SS Delta)^-1),
// <c_p c_q> = -i Gamma_out, weights lambda_a^* lambda_b <B_b|B_a> r_ab / S.
// Per ordered pair (a, b) of the chain's superposition: om = lambda_a^* lambda_b <B_b|B_a> r_ab,
// rho = <B_b|B_a> r_ab (when s_rho is given), the patch set S and Y_ab = Delta (1 + G_SS Delta)^-1,
// so that M_ab^-1 = G + G_S Y_ab G_S^T on the rows and columns used (G antisymmetric).
template <typename T>
__device__ inline void pair_setup(const LaunchCtx &lc, int c, const ChainDev &ch, const TensorDev &Tn, const T *G,
                                  const int8_t *lk, double2 (*s_Y)[64], double2 *s_om, double2 *s_rho,
                                  int (*s_S)[8], int *s_s, double2 *s_work) {
  const int n = ch.n, L = ch.L, K = ch.K, group = ch.group;
  const int npairs = K * K;
  // per ordered pair: r_ab and Y_ab = Delta (1 + G_SS Delta)^-1, four pairs at a time
  for (int p0 = 0; p0 < npairs; p0 += 4) {
    const int pr = p0 + threadIdx.x;
    if (threadIdx.x < 4 && pr < npairs) {
      const int a = pr / K, b = pr % K;
      double2 r = make_double2(1.0, 0.0);
      int s = 0;
      if (!(a == 0 && b == 0)) {
        PatchSet ps;
        double2 *W = s_work + threadIdx.x * (kPairLd * kPairLd + 64);
        double2 *C = W + kPairLd * kPairLd;
        build_pair_matrix(Tn, a, b, L, group, plain_view(G, n), lk, nullptr, nullptr, -1, 0, W, ps);
        s = ps.s;
        for (int i = 0; i < s; ++i)
          for (int j = 0; j < s; ++j) {
            double2 v = make_double2(i == j ? 1.0 : 0.0, 0.0);
            for (int q = 0; q < s; ++q) v = cadd(v, cscale(W[(s + q) * kPairLd + s + j], W[i * kPairLd + q].x));
            C[i * 8 + j] = v;
          }
        int piv[8];
        if (!ggf_cinvert(C, s, 8, piv)) lc.flags[c] |= GGF_FLAG_NONFINITE;
        for (int i = 0; i < s; ++i)
          for (int j = 0; j < s; ++j) {
            double2 v = make_double2(0.0, 0.0);
            for (int q = 0; q < s; ++q) v = cadd(v, cmul(W[(s + i) * kPairLd + s + q], C[q * 8 + j]));
            s_Y[pr][i * 8 + j] = v;
          }
        for (int q = 0; q < s; ++q) s_S[pr][q] = ps.idx[q];
        r = pair_ratio(W, s);
      }
      s_s[pr] = s;
      s_om[pr] = cmul(Tn.w[a][b], r);
      if (s_rho) s_rho[pr] = cmul(Tn.ov[a][b], r);
    }
  }
  __syncthreads();
}

// b G_xy b^T on the 2x2 physical block of sites (x, y), plus the on-site block a when x == y.
template <typename T>
__device__ inline void out_base(const T *G, int n, const TensorDev &Tn, int x, int y, double base[4]) {
  base[0] = base[1] = base[2] = base[3] = 0.0;
  for (int i = 0; i < 8; ++i) {
    const T *grow = G + static_cast<size_t>(8 * x + i) * n + 8 * y;
    double t0 = 0.0, t1 = 0.0;
    for (int j = 0; j < 8; ++j) {
      const double g = static_cast<double>(grow[j]);
      t0 += g * Tn.b[0 * 8 + j];
      t1 += g * Tn.b[1 * 8 + j];
    }
    base[0] += Tn.b[0 * 8 + i] * t0;
    base[1] += Tn.b[0 * 8 + i] * t1;
    base[2] += Tn.b[1 * 8 + i] * t0;
    base[3] += Tn.b[1 * 8 + i] * t1;
  }
  if (x == y) {
    base[0] += Tn.a[0]; base[1] += Tn.a[1]; base[2] += Tn.a[2]; base[3] += Tn.a[3];
  }
}

// Gamma_out of one pair on the block (x, y): base + v_x Y v_y^T, v_x[p][q] = b_p . G[x-block, S_q]
// (G_Sy = -G_yS^T turns -G_xS Y G_Sy into + v_x Y v_y^T).
template <typename T>
__device__ inline void out_pair(const T *G, int n, const TensorDev &Tn, int x, int y, int s, const int *S,
                                const double2 *Y, const double base[4], double2 gm[4]) {
  for (int q = 0; q < 4; ++q) gm[q] = make_double2(base[q], 0.0);
  if (s == 0) return;
  double vx[2][8], vy[2][8];
  for (int q = 0; q < s; ++q) {
    const int col = S[q];
    double ax0 = 0, ax1 = 0, ay0 = 0, ay1 = 0;
    for (int i = 0; i < 8; ++i) {
      const double gx = static_cast<double>(G[static_cast<size_t>(8 * x + i) * n + col]);
      const double gy = static_cast<double>(G[static_cast<size_t>(8 * y + i) * n + col]);
      ax0 += Tn.b[i] * gx; ax1 += Tn.b[8 + i] * gx;
      ay0 += Tn.b[i] * gy; ay1 += Tn.b[8 + i] * gy;
    }
    vx[0][q] = ax0; vx[1][q] = ax1; vy[0][q] = ay0; vy[1][q] = ay1;
  }
  for (int pp = 0; pp < 2; ++pp)
    for (int qq = 0; qq < 2; ++qq) {
      double2 v = make_double2(0, 0);
      for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) v = cadd(v, cscale(Y[i * 8 + j], vx[pp][i] * vy[qq][j]));
      gm[pp * 2 + qq] = cadd(gm[pp * 2 + qq], v);
    }
}

// <phi_x^+ phi_y> (x != y) from Gamma_out on the block (x, y): phi = (c_0 + i c_1)/2,
// <c_p c_q> = -i Gamma_pq, so 1/4 [<c0c0> + i<c0c1> - i<c1c0> + <c1c1>].
__device__ inline double2 hop_xy(const double2 gm[4]) {
  const double2 m00 = make_double2(gm[0].y, -gm[0].x), m01 = make_double2(gm[1].y, -gm[1].x);
  const double2 m10 = make_double2(gm[2].y, -gm[2].x), m11 = make_double2(gm[3].y, -gm[3].x);
  double2 bil = cadd(m00, m11);
  bil = cadd(bil, make_double2(-m01.y, m01.x));
  bil = csub(bil, make_double2(-m10.y, m10.x));
  return cscale(bil, 0.25);
}

// <phi_y^+ phi_x> from the same block: <c_{y b} c_{x a}> = -i Gamma[y b][x a] = +i Gamma[x a][y b].
__device__ inline double2 hop_yx(const double2 gm[4]) {
  // 1/4 [<cy0 cx0> + i<cy0 cx1> - i<cy1 cx0> + <cy1 cx1>]
  const double2 m00 = make_double2(-gm[0].y, gm[0].x), m10 = make_double2(-gm[2].y, gm[2].x);
  const double2 m01 = make_double2(-gm[1].y, gm[1].x), m11 = make_double2(-gm[3].y, gm[3].x);
  double2 bil = cadd(m00, m11);
  bil = cadd(bil, make_double2(-m10.y, m10.x));      // + i <cy0 cx1> = + i m10 (Gamma[x1][y0])
  bil = csub(bil, make_double2(-m01.y, m01.x));      // - i <cy1 cx0> = - i m01 (Gamma[x0][y1])
  return cscale(bil, 0.25);
}

// G on the 4 Majoranas of link ell (antisymmetric 4x4 from six entries).
template <typename T>
__device__ inline void link_block(const T *G, int n, const int u[4], double gu[16]) {
  using V2 = typename Vec2<T>::type;
  const V2 r0 = *reinterpret_cast<const V2 *>(G + static_cast<size_t>(u[0]) * n + u[2]);
  const V2 r1 = *reinterpret_cast<const V2 *>(G + static_cast<size_t>(u[1]) * n + u[2]);
  const double g01 = static_cast<double>(G[static_cast<size_t>(u[0]) * n + u[1]]);
  const double g23 = static_cast<double>(G[static_cast<size_t>(u[2]) * n + u[3]]);
  const double v[16] = {0.0, g01, static_cast<double>(r0.x), static_cast<double>(r0.y),
                        -g01, 0.0, static_cast<double>(r1.x), static_cast<double>(r1.y),
                        -static_cast<double>(r0.x), -static_cast<double>(r1.x), 0.0, g23,
                        -static_cast<double>(r0.y), -static_cast<double>(r1.y), -g23, 0.0};
#pragma unroll
  for (int q = 0; q < 16; ++q) gu[q] = v[q];
}

// Mixed occupation X_ab of link ell's outgoing mode (Sec. 5.3):
// X = en + (1/2) tr(M_ab^-1[U,U] O eq O^T), M_ab^-1[U,U] = G_UU + G_US Y G_US^T.
template <typename T>
__device__ inline double2 mixed_occupation(const T *G, int n, const TensorDev &Tn, int a, int b, int ell, int kv,
                                           int group, const int u[4], const double gu[16], int s, const int *S,
                                           const double2 *Y) {
  double2 gm[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) gm[q] = make_double2(gu[q], 0.0);
  if (s > 0) {
    double vs[4][8];
    for (int i = 0; i < 4; ++i)
      for (int q = 0; q < s; ++q) vs[i][q] = static_cast<double>(G[static_cast<size_t>(u[i]) * n + S[q]]);
    for (int i = 0; i < 4; ++i) {
      double2 vy[8];   // (G_US Y)[i][q]
      for (int q = 0; q < s; ++q) {
        double2 v = make_double2(0.0, 0.0);
        for (int p = 0; p < s; ++p) v = cadd(v, cscale(Y[p * 8 + q], vs[i][p]));
        vy[q] = v;
      }
      for (int j = 0; j < 4; ++j) {
        double2 v = make_double2(0.0, 0.0);
        for (int q = 0; q < s; ++q) v = cadd(v, cscale(vy[q], vs[j][q]));
        gm[i * 4 + j] = cadd(gm[i * 4 + j], v);
      }
    }
  }
  const double2 *eq = Tn.eq0;
  double2 x = Tn.en0;
  for (int l = 0; l < Tn.nl[a][b]; ++l)
    if (Tn.lk[a][b][l] == ell) { eq = Tn.eq[a][b][l]; x = Tn.en[a][b][l]; }
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    double2 row[4];
    rotate_dg_row(eq, kv, group, jj, row);     // row jj of O eq O^T
#pragma unroll
    for (int i = 0; i < 4; ++i) x = cadd(x, cscale(cmul(gm[i * 4 + jj], row[i]), 0.5));
  }
  return x;
}

template <typename T, bool EL_ONLY>
__device__ __forceinline__ void measure_chain(const LaunchCtx &lc, uint32_t mask, double *out) {
  __shared__ double2 s_Y[16][64];
  __shared__ double2 s_om[16];
  __shared__ int s_S[16][8];
  __shared__ int s_s[16];
  __shared__ double red[8];
  extern __shared__ double2 s_work[];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, K = ch.K, group = ch.group;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  const int npairs = K * K;
  pair_setup<T>(lc, c, ch, Tn, G, lk, s_Y, s_om, nullptr, s_S, s_s, s_work);
  __syncthreads();
  double Sv = 0.0;
  for (int p = 0; p < npairs; ++p) Sv += s_om[p].x;
  const double invS = 1.0 / Sv;
  double acc[GGF_NOBS_DEV];
  for (int q = 0; q < GGF_NOBS_DEV; ++q) acc[q] = 0.0;
  const int nmes = min(L / 2, GGF_MAX_MESON);
  for (int x = threadIdx.x; !EL_ONLY && x < V; x += blockDim.x) {
    if (mask & 1u) {
      const int x1 = ggf_shift(x, L, 1, 0), x2 = ggf_shift(x, L, 0, 1);
      double2 z = cmul(link_phase(lk[2 * x], group), link_phase(lk[2 * x1 + 1], group));
      z = cmul(z, cconj(link_phase(lk[2 * x2], group)));
      z = cmul(z, cconj(link_phase(lk[2 * x + 1], group)));
      acc[0] += z.x;
      double2 w = make_double2(1.0, 0.0);
      int p = x;
      for (int t = 0; t < 2; ++t) { w = cmul(w, link_phase(lk[2 * p], group)); p = ggf_shift(p, L, 1, 0); }
      for (int t = 0; t < 2; ++t) { w = cmul(w, link_phase(lk[2 * p + 1], group)); p = ggf_shift(p, L, 0, 1); }
      for (int t = 0; t < 2; ++t) { p = ggf_shift(p, L, -1, 0); w = cmul(w, cconj(link_phase(lk[2 * p], group))); }
      for (int t = 0; t < 2; ++t) { p = ggf_shift(p, L, 0, -1); w = cmul(w, cconj(link_phase(lk[2 * p + 1], group))); }
      acc[1] += w.x;
    }
    if (mask & 6u) {
      // v_x[pair][p][q] = b_p . G[x-block, S_pair q]; base terms b_p G_xy b_q^T computed on the fly
      for (int r = 0; r <= ((mask & 4u) ? nmes : 0); ++r) {
        if (r == 0 && !(mask & 2u)) continue;
        const int y = (r == 0) ? x : ggf_shift(x, L, r, 0);
        double base[4];   // (b G_xy b^T)[p][q] (+ a on site)
        out_base(G, n, Tn, x, y, base);
        double2 tot = make_double2(0.0, 0.0);
        for (int pr = 0; pr < npairs; ++pr) {
          double2 gm[4];
          out_pair(G, n, Tn, x, y, s_s[pr], s_S[pr], s_Y[pr], base, gm);
          double2 f;
          if (r == 0) f = cscale(cadd(make_double2(1.0, 0.0), gm[1]), 0.5);    // (1 + Gamma_out[x0,x1]) / 2
          else f = cscale(hop_xy(gm), 2.0);                                      // 2 <phi_x^+ phi_y>
          tot = cadd(tot, cmul(s_om[pr], f));
        }
        if (r == 0) {
          acc[2] += tot.x * invS;
        } else {
          double2 line = make_double2(1.0, 0.0);
          int p = x;
          for (int t = 0; t < r; ++t) { line = cmul(line, link_phase(lk[2 * p], group)); p = ggf_shift(p, L, 1, 0); }
          acc[4 + r - 1] += cmul(line, tot).x * invS;
        }
      }
    }
  }
  if (EL_ONLY || (mask & 8u)) {
    // Electric field per link (Sec. 5.3), lattice mean of Re f_E with e_0 = 0, e_j = 1:
    // f_E = sum_ab om_ab X_ab / S, X_ab = en + (1/2) tr(M_ab^-1[U,U] O eq O^T) the mixed
    // occupation of the link's outgoing mode, M_ab^-1[U,U] = G_UU + G_US Y_ab G_US^T.
    // The six entries of the antisymmetric G_UU: (u0,u1) and (u2,u3) on the sites' diagonal
    // blocks, (u0|u1, u2..u3) as two aligned pairs (u2 is even).
    for (int ell = threadIdx.x; ell < 2 * V; ell += blockDim.x) {
      int u[4];
      ggf_link_u(ell, L, u);
      double gu[16];
      link_block(G, n, u, gu);
      const int kv = lk[ell];
      double2 tot = make_double2(0.0, 0.0);
      for (int pr = 0; pr < npairs; ++pr)
        tot = cadd(tot, cmul(s_om[pr], mixed_occupation(G, n, Tn, pr / K, pr % K, ell, kv, group, u, gu, s_s[pr],
                                                        s_S[pr], s_Y[pr])));
      acc[GGF_NOBS_DEV - 1] += 0.5 * tot.x * invS;   // two links per site
    }
  }
  if (EL_ONLY) {
    const double t = block_sum(acc[GGF_NOBS_DEV - 1], red);
    if (threadIdx.x == 0)
      for (int q = 0; q < GGF_NOBS_DEV; ++q)
        out[static_cast<size_t>(c) * GGF_NOBS_DEV + q] = (q == GGF_NOBS_DEV - 1) ? t / V : 0.0;
    return;
  }
  for (int q = 0; q < GGF_NOBS_DEV; ++q) {
    const double t = block_sum(acc[q], red);
    if (threadIdx.x == 0) out[static_cast<size_t>(c) * GGF_NOBS_DEV + q] = t / V;
  }
  if (threadIdx.x == 0) out[static_cast<size_t>(c) * GGF_NOBS_DEV + 3] =
      (!EL_ONLY && (mask & 2u)) ? lc.logw[c] + (K > 1 ? log(Sv) : 0.0) : 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_measure(LaunchCtx lc, uint32_t mask, double *out) {
  measure_chain<T, false>(lc, mask, out);
}

// Electric-field slot only (the other slots written as 0).
template <typename T>
__global__ __launch_bounds__(128) void k_electric(LaunchCtx lc, double *out) {
  measure_chain<T, true>(lc, 8u, out);
}

// Electric-field slot only when every chain has K = 1: f_E = Re X with
// X = en0 + (1/2) tr(G_UU R_k) = en0 + sum_{i<j} G_UU[i][j] R_k[j][i] (G_UU and R_k
// antisymmetric), R_k = O_k eq0 O_k^T for link value k, one table per workgroup.
template <typename T>
__global__ __launch_bounds__(128) void k_electric1(LaunchCtx lc, double *out) {
  __shared__ double s_R[GGF_ZN_MAX][16];
  __shared__ double red[2];
  using V2 = typename Vec2<T>::type;
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, group = ch.group;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  for (int te = threadIdx.x; te < 16 * group; te += blockDim.x) {
    // entry e of Re(O_k eq0 O_k^T), unrolled with constant indices (no private-array scratch)
    const int k = te >> 4, e = te & 15;
    double co = 1.0, si = 0.0;
    if (k != 0) {
      if (group == 2) co = -1.0;
      else sincospi(2.0 * k / group, &si, &co);
    }
    const double o[4][4] = {{co, si, 0.0, 0.0}, {-si, co, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}, {0.0, 0.0, 0.0, 1.0}};
    double q[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) q[i] = Tn.eq0[i].x;
    double val = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) v += o[i][a] * q[a * 4 + b] * o[j][b];
        if (i * 4 + j == e) val = v;
      }
    s_R[k][e] = val;
  }
  __syncthreads();
  double acc = 0.0;
  for (int ell = threadIdx.x; ell < 2 * V; ell += blockDim.x) {
    int u[4];
    ggf_link_u(ell, L, u);
    const V2 r0 = *reinterpret_cast<const V2 *>(G + static_cast<size_t>(u[0]) * n + u[2]);
    const V2 r1 = *reinterpret_cast<const V2 *>(G + static_cast<size_t>(u[1]) * n + u[2]);
    const double g01 = static_cast<double>(G[static_cast<size_t>(u[0]) * n + u[1]]);
    const double g23 = static_cast<double>(G[static_cast<size_t>(u[2]) * n + u[3]]);
    const double *R = s_R[lk[ell]];
    acc += Tn.en0.x + g01 * R[1 * 4 + 0] + static_cast<double>(r0.x) * R[2 * 4 + 0] +
           static_cast<double>(r0.y) * R[3 * 4 + 0] + static_cast<double>(r1.x) * R[2 * 4 + 1] +
           static_cast<double>(r1.y) * R[3 * 4 + 1] + g23 * R[3 * 4 + 2];
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0)
    for (int q = 0; q < GGF_NOBS_DEV; ++q)
      out[static_cast<size_t>(c) * GGF_NOBS_DEV + q] = (q == GGF_NOBS_DEV - 1) ? 0.5 * t / V : 0.0;
}


// Local energy of the gauged Hamiltonian (Sec. 2 hopping with the link phase D(g) and the
// pi-flux signs, chemical and staggered mass terms; Sec. 2.3 plaquette; Sec. 5.3 electric
// term) per chain, with the pair matrices of the linear variational step for lambda:
//   h_ab = transition expectation of H in the pair (a, b) (Sec. 5.2, 5.3),
//   out[0] = Re sum_ab om_ab h_ab / S, out[1 + 4 p ..] = rho_p / S and rho_p h_p / S
//   (complex, p = a K + b), rho_ab = <B_b|B_a> r_ab; the other entries 0.
template <typename T>
__global__ __launch_bounds__(256) void k_energy(LaunchCtx lc, EnergyCp cp, double *out) {
  __shared__ double2 s_Y[16][64];
  __shared__ double2 s_om[16], s_rho[16], s_h[16];
  __shared__ int s_S[16][8];
  __shared__ int s_s[16];
  __shared__ double red[8];
  extern __shared__ double2 s_work[];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, K = ch.K, group = ch.group;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  const int npairs = K * K;
  pair_setup<T>(lc, c, ch, Tn, G, lk, s_Y, s_om, s_rho, s_S, s_s, s_work);
  for (int pr = 0; pr < npairs; ++pr) {
    const int a = pr / K, b = pr % K, s = s_s[pr];
    double hr = 0.0, hi = 0.0;
    for (int x = threadIdx.x; x < V; x += blockDim.x) {
      const int x2 = x / L;
      double2 h = make_double2(0.0, 0.0);
      double base[4];
      double2 gm[4];
      // chemical + staggered mass: <phi_x^+ phi_x> = (1 + Gamma_out[x0,x1]) / 2
      out_base(G, n, Tn, x, x, base);
      out_pair(G, n, Tn, x, x, s, s_S[pr], s_Y[pr], base, gm);
      const double sgn = (((x % L) + x2) & 1) ? -1.0 : 1.0;
      h = cadd(h, cscale(cscale(cadd(make_double2(1.0, 0.0), gm[1]), 0.5), cp.mu + sgn * cp.m));
      for (int mu = 0; mu < 2; ++mu) {
        const int ell = 2 * x + mu;
        const int y = mu == 0 ? ggf_shift(x, L, 1, 0) : ggf_shift(x, L, 0, 1);
        // hopping: i eta D <phi_x^+ phi_y> - i eta D^* <phi_y^+ phi_x>, eta = -1 on horizontal
        // links of odd rows
        out_base(G, n, Tn, x, y, base);
        out_pair(G, n, Tn, x, y, s, s_S[pr], s_Y[pr], base, gm);
        const double2 D = link_phase(lk[ell], group);
        const double te = (mu == 0 && (x2 & 1)) ? -cp.t : cp.t;
        const double2 f = cmul(D, hop_xy(gm));
        const double2 g = cmul(cconj(D), hop_yx(gm));
        h = cadd(h, cscale(make_double2(g.y - f.y, f.x - g.x), te));   // i (f - g)
        if (cp.ke != 0.0) {
          int u[4];
          ggf_link_u(ell, L, u);
          double gu[16];
          link_block(G, n, u, gu);
          h = cadd(h, cscale(mixed_occupation(G, n, Tn, a, b, ell, lk[ell], group, u, gu, s, s_S[pr], s_Y[pr]),
                             cp.ke));
        }
      }
      if (cp.kb != 0.0) {
        const int x1n = ggf_shift(x, L, 1, 0), x2n = ggf_shift(x, L, 0, 1);
        double2 z = cmul(link_phase(lk[2 * x], group), link_phase(lk[2 * x1n + 1], group));
        z = cmul(z, cconj(link_phase(lk[2 * x2n], group)));
        z = cmul(z, cconj(link_phase(lk[2 * x + 1], group)));
        h.x += 2.0 * cp.kb * z.x;                                     // kb (U + U^*)
      }
      hr += h.x;
      hi += h.y;
    }
    const double tr = block_sum(hr, red);
    const double ti = block_sum(hi, red);
    if (threadIdx.x == 0) s_h[pr] = make_double2(tr, ti);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double Sv = 0.0, e = 0.0;
    for (int p = 0; p < npairs; ++p) {
      Sv += s_om[p].x;
      e += cmul(s_om[p], s_h[p]).x;
    }
    const double invS = 1.0 / Sv;
    double *o = out + static_cast<size_t>(c) * GGF_ENERGY_STRIDE_DEV;
    for (int q = 0; q < GGF_ENERGY_STRIDE_DEV; ++q) o[q] = 0.0;
    for (int p = 0; p < npairs; ++p) {
      const double2 rh = cmul(s_rho[p], s_h[p]);
      o[1 + 4 * p] = s_rho[p].x * invS;
      o[2 + 4 * p] = s_rho[p].y * invS;
      o[3 + 4 * p] = rh.x * invS;
      o[4 + 4 * p] = rh.y * invS;
    }
    o[0] = e * invS;
    if (!isfinite(o[0])) lc.flags[c] |= GGF_FLAG_NONFINITE;
  }
}

// Rows for the gradient with respect to the patch bond states (one workgroup per chain).  S is
// the union of the patch links' Majoranas (ascending).  The part of the local energy linear in
// X = M^-1 is sum_ij C_ij X_ij: the bilinear <phi_x^+ phi_y> (coefficient beta) contributes
// -(beta / 4) i conj(z_p) z_q at X[8x + p][8y + q], z = b_0 + i b_1 (the rows of the
// physical-virtual block), and the mixed occupation of link l with the reference bond's response,
// X_l = en0 + (1/2) tr(X_UU O eq0 O^T), contributes (ke / 2) (O eq0 O^T)_ji at X[u_i][u_j].
// With G real antisymmetric, V_b(y) = sum_q z_q G[S_b][8y + q] gives
//   R[a][b] = sum_ij C_ij G[i][S_a] G[S_b][j]
//           = (i / 4) sum beta_xy conj(V_a(x)) V_b(y) - (ke / 2) sum_l sum_ij Q_ji G[S_a][u_i] G[S_b][u_j].
// V lives in LDS (s L^2 <= 4096 complex), O eq0 O^T per group element in a table.
template <typename T>
__global__ __launch_bounds__(256) void k_bond_rows(LaunchCtx lc, EnergyCp cp, double *out) {
  __shared__ double2 s_v[4096];
  __shared__ double2 s_q[GGF_ZN_MAX][16];
  __shared__ int s_S[12];
  __shared__ int s_s;
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, K = ch.K, group = ch.group;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  double *o = out + static_cast<size_t>(c) * GGF_BOND_STRIDE_DEV;
  if (threadIdx.x == 0) {
    int m = 0;
    for (int k = 1; k < K; ++k) {
      int u[4];
      ggf_link_u(Tn.lk[k][0][0], L, u);
      for (int i = 0; i < 4; ++i) {
        bool seen = false;
        for (int q = 0; q < m; ++q) seen = seen || s_S[q] == u[i];
        if (!seen) s_S[m++] = u[i];
      }
    }
    for (int i = 1; i < m; ++i)          // ascending
      for (int j = i; j > 0 && s_S[j - 1] > s_S[j]; --j) {
        const int t = s_S[j];
        s_S[j] = s_S[j - 1];
        s_S[j - 1] = t;
      }
    s_s = m;
  }
  for (int g = threadIdx.x; g < group * 4; g += blockDim.x) {
    double2 row[4];
    rotate_dg_row(Tn.eq0, g / 4, group, g % 4, row);   // row (g % 4) of O(g / 4) eq0 O(g / 4)^T
    for (int j = 0; j < 4; ++j) s_q[g / 4][(g % 4) * 4 + j] = row[j];
  }
  __syncthreads();
  const int s = s_s;
  for (int q = threadIdx.x; q < GGF_BOND_STRIDE_DEV; q += blockDim.x) o[q] = 0.0;
  __syncthreads();
  if (s == 0) return;
  for (int t = threadIdx.x; t < s * V; t += blockDim.x) {
    const int b = t / V, y = t % V;
    const T *row = G + static_cast<size_t>(s_S[b]) * n + 8 * y;
    double2 v = make_double2(0.0, 0.0);
    for (int q = 0; q < 8; ++q) {
      const double gq = static_cast<double>(row[q]);
      v = cadd(v, make_double2(Tn.b[q] * gq, Tn.b[8 + q] * gq));
    }
    s_v[b * V + y] = v;
  }
  __syncthreads();
  const int a = threadIdx.x / s, b = threadIdx.x % s;
  if (threadIdx.x < s * s) {
    const double2 *va = s_v + a * V, *vb = s_v + b * V;
    double2 fer = make_double2(0.0, 0.0), el = make_double2(0.0, 0.0);
    for (int x = 0; x < V; ++x) {
      const int x2 = x / L;
      const double sgn = (((x % L) + x2) & 1) ? -1.0 : 1.0;
      fer = cadd(fer, cscale(cmul(cconj(va[x]), vb[x]), cp.mu + sgn * cp.m));
      for (int mu = 0; mu < 2; ++mu) {
        const int ell = 2 * x + mu;
        const int y = mu == 0 ? ggf_shift(x, L, 1, 0) : ggf_shift(x, L, 0, 1);
        const double2 D = link_phase(lk[ell], group);
        const double te = (mu == 0 && (x2 & 1)) ? -cp.t : cp.t;
        // beta_xy = i te D on <phi_x^+ phi_y>, beta_yx = -i te D^* on <phi_y^+ phi_x>
        const double2 bxy = make_double2(-te * D.y, te * D.x), byx = make_double2(-te * D.y, -te * D.x);
        fer = cadd(fer, cmul(bxy, cmul(cconj(va[x]), vb[y])));
        fer = cadd(fer, cmul(byx, cmul(cconj(va[y]), vb[x])));
        if (cp.ke != 0.0) {
          int u[4];
          ggf_link_u(ell, L, u);
          double ga[4], gb[4];
          for (int i = 0; i < 4; ++i) {
            ga[i] = static_cast<double>(G[static_cast<size_t>(s_S[a]) * n + u[i]]);
            gb[i] = static_cast<double>(G[static_cast<size_t>(s_S[b]) * n + u[i]]);
          }
          const double2 *Q = s_q[lk[ell]];
          for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) el = cadd(el, cscale(Q[j * 4 + i], ga[i] * gb[j]));
        }
      }
    }
    // R = (i / 4) fer - (ke / 2) el
    const double2 r = make_double2(-0.25 * fer.y - 0.5 * cp.ke * el.x, 0.25 * fer.x - 0.5 * cp.ke * el.y);
    o[18 + 2 * (12 * a + b)] = r.x;
    o[19 + 2 * (12 * a + b)] = r.y;
    o[306 + 12 * a + b] = static_cast<double>(G[static_cast<size_t>(s_S[a]) * n + s_S[b]]);
  }
  if (threadIdx.x == 0) {
    o[0] = s;
    o[1] = L;
    for (int q = 0; q < s; ++q) o[2 + q] = s_S[q];
    for (int k = 1; k < K; ++k) o[14 + k] = lk[Tn.lk[k][0][0]];
  }
}

// Real part of Re(coef * Wc), Wc = (1/4) [[-i, 1], [-1, -i]]: the coefficient block of
// Gamma_out[2x + a][2y + b] in coef <phi_x^+ phi_y> (with <c_p c_q> = -i Gamma_pq).
__device__ inline void coef_block(double2 coef, double o[4]) {
  o[0] = 0.25 * coef.y;
  o[1] = 0.25 * coef.x;
  o[2] = -0.25 * coef.x;
  o[3] = 0.25 * coef.y;
}

// The five bilinear terms of H that involve site x: term 0 on-site (x, x), terms 1 + 2 mu
// the hop (x, x + mu), terms 2 + 2 mu the reverse (x + mu, x); (row site, column site, complex
// coefficient of <phi_w^+ phi_y>), with D the phase of the term's link (unused by term 0).
__device__ inline double2 h_coef_d(const EnergyCp &cp, int L, int x, int term, double2 D, int &w, int &y) {
  if (term == 0) {
    const int sgn = (((x % L) + x / L) & 1) ? -1 : 1;
    w = y = x;
    return make_double2(cp.mu + sgn * cp.m, 0.0);
  }
  const int mu = (term - 1) >> 1;
  const int xn = mu == 0 ? ggf_shift(x, L, 1, 0) : ggf_shift(x, L, 0, 1);
  const double te = (mu == 0 && ((x / L) & 1)) ? -cp.t : cp.t;
  if ((term & 1) == 1) {           // t i eta D <phi_x^+ phi_xn>
    w = x;
    y = xn;
    return make_double2(-te * D.y, te * D.x);
  }
  w = xn;                          // -t i eta D^* <phi_xn^+ phi_x>
  y = x;
  return make_double2(-te * D.y, -te * D.x);
}

// The same with the link phase taken from the link field.
__device__ inline double2 h_coef(const EnergyCp &cp, const int8_t *lk, int L, int group, int x, int term, int &w,
                                 int &y) {
  const double2 D = term == 0 ? make_double2(1.0, 0.0) : link_phase(lk[2 * x + ((term - 1) >> 1)], group);
  return h_coef_d(cp, L, x, term, D, w, y);
}

// The same terms as coefficient blocks of Gamma_out[2w + a][2y + b].
__device__ inline void h_term(const EnergyCp &cp, const int8_t *lk, int L, int group, int x, int term, int &w,
                              int &y, double o[4]) {
  coef_block(h_coef(cp, lk, L, group, x, term, w, y), o);
}

// Rotated electric response R_k = O_k eq0 O_k^T (real part) for every link value k, 16 doubles each.
__device__ inline void sens_r_table(const TensorDev &Tn, int group, double *s_R) {
  const int tid = threadIdx.x;
  for (int te = tid; te < 16 * group; te += blockDim.x) {
    const int k = te >> 4, e = te & 15;
    double co = 1.0, si = 0.0;
    if (k != 0) {
      if (group == 2) co = -1.0;
      else sincospi(2.0 * k / group, &si, &co);
    }
    const double o[4][4] = {{co, si, 0.0, 0.0}, {-si, co, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}, {0.0, 0.0, 0.0, 1.0}};
    double q[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) q[i] = Tn.eq0[i].x;
    double val = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) v += o[i][a] * q[a * 4 + b] * o[j][b];
        if (i * 4 + j == e) val = v;
      }
    s_R[k * 16 + e] = val;
  }
}

// a-block, b-block and S_N of the K = 1 sensitivities: per site the rows of G on the 5
// neighbouring blocks (accumulated into s_Sa, s_Sb, s_SN by LDS atomics).  Only the first wave
// takes part, so that the atomics of each sum come in a fixed order (rows reproducible bit for bit).
template <typename T>
__device__ inline void sens_sites(const EnergyCp &cp, const int8_t *lk, int L, int group, const T *G, int n,
                                  const TensorDev &Tn, double *s_Sa, double *s_Sb, double *s_SN) {
  const int V = L * L, tid = threadIdx.x;
  if (tid >= 64) return;
  for (int x = tid; x < V; x += 64) {
    double sb[16];
    for (int q = 0; q < 16; ++q) sb[q] = 0.0;
    {
      // a-block: the on-site term's block, transposed
      int w, y;
      double o[4];
      h_term(cp, lk, L, group, x, 0, w, y, o);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) atomicAdd(&s_Sa[b * 2 + a], o[a * 2 + b]);
    }
    // blocks with row site x: (x, y) for y = x, x + mu (hop) and x - mu (reverse of the hop into x)
    // blocks with column site x: (w, x) for w = x, x - mu (hop) and x + mu (reverse)
    for (int nb = 0; nb < 5; ++nb) {
      // neighbour y of x and the blocks (x, y) and (y, x) among the terms of x and of x - mu
      int y = x;
      if (nb == 1) y = ggf_shift(x, L, 1, 0);
      if (nb == 2) y = ggf_shift(x, L, 0, 1);
      if (nb == 3) y = ggf_shift(x, L, -1, 0);
      if (nb == 4) y = ggf_shift(x, L, 0, -1);
      // L = 2: x - mu is x + mu, whose blocks nb = 1, 2 already collected (from both owners)
      if ((nb == 3 && y == ggf_shift(x, L, 1, 0)) || (nb == 4 && y == ggf_shift(x, L, 0, 1))) continue;
      double orow[4] = {0, 0, 0, 0}, ocol[4] = {0, 0, 0, 0};   // blocks (x, y) and (y, x)
      const int owners[2] = {x, y};
      for (int oi = 0; oi < (nb == 0 ? 1 : 2); ++oi)
        for (int term = 0; term < 5; ++term) {
          int w2, y2;
          double o[4];
          h_term(cp, lk, L, group, owners[oi], term, w2, y2, o);
          if (nb == 0 && term != 0) continue;
          if (nb != 0 && term == 0) continue;
          if (w2 == x && y2 == y)
            for (int q = 0; q < 4; ++q) orow[q] += o[q];
          if (w2 == y && y2 == x)
            for (int q = 0; q < 4; ++q) ocol[q] += o[q];
        }
      if (nb == 0) {
        for (int q = 0; q < 4; ++q) ocol[q] = orow[q];
      }
      for (int i = 0; i < 8; ++i) {
        const T *grow = G + static_cast<size_t>(8 * x + i) * n + 8 * y;
        double t0 = 0.0, t1 = 0.0;   // T[i][y][beta] = sum_j G[8x+i][8y+j] b[beta][j]
        for (int j = 0; j < 8; ++j) {
          const double g = static_cast<double>(grow[j]);
          t0 += g * Tn.b[j];
          t1 += g * Tn.b[8 + j];
        }
        for (int a = 0; a < 2; ++a) {
          // dB G B^T: Sb[a][i] += sum_beta C[x a][y beta] T[i][y][beta]
          sb[a * 8 + i] += orow[a * 2 + 0] * t0 + orow[a * 2 + 1] * t1;
          // B G dB^T: Sb[b][i] -= sum_alpha C[y alpha][x b] T[i][y][alpha]
          sb[a * 8 + i] -= ocol[0 * 2 + a] * t0 + ocol[1 * 2 + a] * t1;
        }
      }
    }
    for (int q = 0; q < 16; ++q) atomicAdd(&s_Sb[q], sb[q]);
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j)
        atomicAdd(&s_SN[i * 8 + j], 0.5 * static_cast<double>(G[static_cast<size_t>(8 * x + i) * n + 8 * x + j]));
  }
}

// Every entry of the sensitivity row but the S_e d-block (thread tid < 100 writes its share).
__device__ inline void sens_write_rest(double *o, const double *s_Sa, const double *s_Sb, const double *s_SN) {
  const int tid = threadIdx.x;
  if (tid < 64) o[100 + (2 + (tid >> 3)) * 10 + 2 + (tid & 7)] = s_SN[tid];
  if (tid < 16) {
    const int a = tid >> 3, i = tid & 7;
    o[(2 + i) * 10 + a] = s_Sb[tid];          // S_e[2 + i][a] = Sb[a][i]
  }
  if (tid < 4) o[(tid >> 1) * 10 + (tid & 1)] = s_Sa[tid];
  if (tid < 20) {
    const int a = tid / 10, j = tid % 10;
    if (j >= 2) o[a * 10 + j] = 0.0;           // S_e[0:2][2:10] = 0
  }
  if (tid < 100) {
    const int i = tid / 10, j = tid % 10;
    if (i < 2 || j < 2) o[100 + tid] = 0.0;    // S_N outside the d-block
  }
}

// Sensitivities of one K = 1 chain to its on-site covariance Gamma_A: for Delta = [E, Gamma_A]
// (E antisymmetric), Re d e(G) = tr(Delta S_e) and d log N(G) = tr(Delta S_N), with the
// transposed-trace convention tr(Delta S) = sum_ij Delta_ij S_ji.  With P = B G, C the
// coefficients of Gamma_out in the local energy and R_k the rotated electric response,
//   S_e[a-block]  = sum_x C[x, x]^T,
//   S_e[b^T-block] from dB G B^T + B G dB^T (rows of G on the 5 neighbouring blocks),
//   S_e[d-block]  = sum_z (P^T C P)[z, z]^T + ke sum_l sum_{i<j} R_k[j][i] G[z, u_j] (x) G[z, u_i],
//   S_N[d-block]  = (1/2) sum_x G[x, x]  (log N = (1/2) log det M + const).
// out[c][0..99] = Re S_e, out[c][100..199] = S_N (row-major 10 x 10).  L <= 32.
// Per row stripe z, the sites are taken in chunks of R whole lattice rows: the Hamiltonian blocks of
// a site x pair it with x, x + e1 (same row) and x + e2 (next row), so U_z is formed on the chunk's
// rows and the row after it, at most kSensSites sites (R = min(L, kSensSites / L - 1)).
constexpr int kSensSites = 448;
template <typename T>
__global__ __launch_bounds__(256) void k_sens(LaunchCtx lc, EnergyCp cp, double *out, int max_sites) {
  extern __shared__ double s_dyn[];
  double *s_U = s_dyn;                       // U_z[i][2 ls + a] = sum_j G[8z+i][8w+j] b[a][j], w the chunk's ls-th site
  __shared__ double s_Sa[4], s_Sb[16], s_SN[64];
  __shared__ double s_R[GGF_ZN_MAX][16];
  __shared__ double s_red[4][64];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, group = ch.group;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  const int tid = threadIdx.x;
  if (tid < 4) s_Sa[tid] = 0.0;
  if (tid < 16) s_Sb[tid] = 0.0;
  if (tid < 64) s_SN[tid] = 0.0;
  sens_r_table(Tn, group, &s_R[0][0]);
  __syncthreads();
  // (1) per site: a-block, b-block and S_N
  sens_sites<T>(cp, lk, L, group, G, n, Tn, s_Sa, s_Sb, s_SN);
  // (2) d-block: per row stripe z, in chunks of R lattice rows
  const int R = min(L, kSensSites / L - 1);
  const int ij = tid & 63, part = tid >> 6;
  const int pi = ij >> 3, pj = ij & 7;
  // index of site s among the chunk's sites (rows r0 .. r0 + nr, the last taken mod L)
  auto local = [&](int s_, int r0) { return (((s_ / L) - r0 + L) % L) * L + s_ % L; };
  double sd = 0.0;
  for (int z = 0; z < V; ++z) {
    double acc = 0.0;
    for (int r0 = 0; r0 < L; r0 += R) {
      const int nr = min(R, L - r0);
      const int ns = (nr + 1) * L;
      __syncthreads();                       // readers of the previous chunk's U_z are done
      for (int e = tid; e < 16 * ns; e += blockDim.x) {
        const int i = e / (2 * ns), col = e % (2 * ns), ls = col >> 1, a = col & 1;
        const int w = ((r0 + ls / L) % L) * L + ls % L;
        const T *grow = G + static_cast<size_t>(8 * z + i) * n + 8 * w;
        double v = 0.0;
        for (int j = 0; j < 8; ++j) v += static_cast<double>(grow[j]) * Tn.b[a * 8 + j];
        s_U[i * 2 * ns + col] = v;
      }
      __syncthreads();
      for (int lx = part; lx < nr * L; lx += 4) {
        const int x = (r0 + lx / L) * L + lx % L;
        for (int term = 0; term < 5; ++term) {
          int w, y;
          double o[4];
          h_term(cp, lk, L, group, x, term, w, y, o);
          const int lw = local(w, r0), ly = local(y, r0);
          const double ui0 = s_U[pi * 2 * ns + 2 * lw], ui1 = s_U[pi * 2 * ns + 2 * lw + 1];
          const double uj0 = s_U[pj * 2 * ns + 2 * ly], uj1 = s_U[pj * 2 * ns + 2 * ly + 1];
          acc += ui0 * (o[0] * uj0 + o[1] * uj1) + ui1 * (o[2] * uj0 + o[3] * uj1);
        }
      }
    }
    if (cp.ke != 0.0)
      for (int ell = part; ell < 2 * V; ell += 4) {
        int u[4];
        ggf_link_u(ell, L, u);
        const double *Rk = s_R[lk[ell]];
        double vp[4], vq[4];   // G[8z + pj][u], G[8z + pi][u] (S_d[pj][pi] collects the sum)
        for (int i = 0; i < 4; ++i) {
          vp[i] = static_cast<double>(G[static_cast<size_t>(8 * z + pj) * n + u[i]]);
          vq[i] = static_cast<double>(G[static_cast<size_t>(8 * z + pi) * n + u[i]]);
        }
        for (int i = 0; i < 4; ++i)
          for (int j = i + 1; j < 4; ++j) acc += cp.ke * Rk[j * 4 + i] * vp[j] * vq[i];
      }
    sd += acc;   // (P^T C P)[z][pi][pj] + electric part; S_d[pj][pi] collects it
  }
  s_red[part][ij] = sd;
  __syncthreads();
  double *o = out + static_cast<size_t>(c) * GGF_SENS_STRIDE_DEV;
  if (tid < 64) {
    const double v = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
    // thread (pi, pj) summed (P^T C P)[pi][pj] for the d-block's transpose: S_d[pj][pi]
    o[(2 + pj) * 10 + 2 + pi] = v;
  }
  sens_write_rest(o, s_Sa, s_Sb, s_SN);
}

// The d-block of k_sens as two contractions per row stripe z (V <= 100, stripe staged):
//   CU[2w + a][p] = sum over the 5 bilinear blocks (w, y) with row site w of C[w a][y b] U_z[p][2y + b],
//   T_z[m][p]     = sum_a b[a][m mod 8] CU[2 (m / 8) + a][p] + ke sum_{j > i} R_l[j][i] G[8z + p][u_j]
//                   (m = u_i of link l; every virtual Majorana belongs to one link),
//   S_d[q][p]    += sum_m G[8z + p][m] T_z[m][q],
// so the Hamiltonian's blocks are evaluated once per (site, row) rather than once per (site, row, column).
// Dynamic LDS: stripe 8 (n + 2), T_z n x 8 (U_z 2V x 8 at its start), CU 2V x 8, R max_group x 16 (float64);
// the 5 V block coefficients (complex), their column sites and the links' Majoranas (int16).
// Launched with 512 threads.
template <typename T>
__global__ __launch_bounds__(512, 4) void k_sens_t(LaunchCtx lc, EnergyCp cp, double *out, int max_sites, int max_group) {
  extern __shared__ double s_dyn[];
  double *s_G = s_dyn;                       // stripe z, 8 rows of pitch n + 2 (rows on distinct banks)
  double *s_T = s_G + 64 * max_sites + 16;   // T_z[m][p]
  double *s_U = s_T;                         // U_z[2w + a][i], dead once CU is formed
  double *s_CU = s_T + 64 * max_sites;       // CU[2w + a][p]
  double *s_R = s_CU + 16 * max_sites;       // R_k, 16 per link value
  double2 *s_cc = reinterpret_cast<double2 *>(s_R + 16 * max_group);   // coefficients of the 5 blocks of row site w
  int16_t *s_cy = reinterpret_cast<int16_t *>(s_cc + 5 * max_sites);  // their column sites
  int16_t *s_lu = s_cy + 5 * max_sites;                              // the 4 Majoranas of each link
  __shared__ double s_Sa[4], s_Sb[16], s_SN[64];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, group = ch.group;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk_g = lc.links + ch.link_off;
  __shared__ int8_t s_lk[200];               // the chain's link values (2V <= 200), read by every stage
  const int8_t *lk = s_lk;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * V; e += blockDim.x) s_lk[e] = lk_g[e];
  if (tid < 4) s_Sa[tid] = 0.0;
  if (tid < 16) s_Sb[tid] = 0.0;
  if (tid < 64) s_SN[tid] = 0.0;
  sens_r_table(Tn, group, s_R);
  __syncthreads();   // s_lk complete before the tables read it
  for (int e = tid; e < 5 * V; e += blockDim.x) {
    // row site w: on site, the hops to w + e1 and w + e2 (terms 1, 3 of w), the reverse hops from
    // w - e1 and w - e2 (terms 2, 4 of those sites)
    const int w = e / 5, t = e - 5 * w;
    int owner = w, term = t;
    if (t == 2) term = 3;
    else if (t == 3) { owner = ggf_shift(w, L, -1, 0); term = 2; }
    else if (t == 4) { owner = ggf_shift(w, L, 0, -1); term = 4; }
    int wr, y;
    s_cc[e] = h_coef(cp, lk, L, group, owner, term, wr, y);
    s_cy[e] = static_cast<int16_t>(y);
  }
  for (int ell = tid; ell < 2 * V; ell += blockDim.x) {
    int u[4];
    ggf_link_u(ell, L, u);
    for (int k = 0; k < 4; ++k) s_lu[4 * ell + k] = static_cast<int16_t>(u[k]);
  }
  __syncthreads();
  sens_sites<T>(cp, lk, L, group, G, n, Tn, s_Sa, s_Sb, s_SN);
  // final contraction: thread = (2 x 2 block of (p, q), one of 32 strided parts of m)
  const int part = tid & 31, blk = tid >> 5;
  const int p0 = 2 * (blk >> 2), q0 = 2 * (blk & 3);
  double sd00 = 0.0, sd01 = 0.0, sd10 = 0.0, sd11 = 0.0;
  // stripe z + 1 is loaded into registers while stripe z is contracted: row r, columns tid + 512 k
  // (n <= 800 for V <= 100, so 2 columns per row and thread)
  const int pitch = n + 2;
  constexpr int kCols = 2;
  double pf[8 * kCols];
  auto load_stripe = [&](int z) {
    const T *src = G + static_cast<size_t>(8 * z) * n;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int k = 0; k < kCols; ++k) {
        const int col = tid + 512 * k;
        pf[r * kCols + k] = col < n ? static_cast<double>(src[static_cast<size_t>(r) * n + col]) : 0.0;
      }
  };
  load_stripe(0);
  for (int z = 0; z < V; ++z) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int k = 0; k < kCols; ++k) {
        const int col = tid + 512 * k;
        if (col < n) s_G[r * pitch + col] = pf[r * kCols + k];
      }
    if (z + 1 < V) load_stripe(z + 1);
    __syncthreads();
    for (int e = tid; e < 16 * V; e += blockDim.x) {
      const int i = e & 7, col = e >> 3, w = col >> 1, a = col & 1;
      const double *grow = s_G + i * pitch + 8 * w;
      double v = 0.0;
      for (int j = 0; j < 8; ++j) v += grow[j] * Tn.b[a * 8 + j];
      s_U[e] = v;                            // U_z[2w + a][i]
    }
    __syncthreads();
    for (int e = tid; e < 8 * V; e += blockDim.x) {
      const int w = e >> 3, p = e & 7;
      double c0 = 0.0, c1 = 0.0;
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        // block coef * (1/4) [[-i, 1], [-1, -i]] (real part), as coef_block
        const double2 cf = s_cc[5 * w + t];
        const int y = s_cy[5 * w + t];
        const double u0 = s_U[(2 * y) * 8 + p], u1 = s_U[(2 * y + 1) * 8 + p];
        c0 += cf.y * u0 + cf.x * u1;
        c1 += cf.y * u1 - cf.x * u0;
      }
      s_CU[(2 * w) * 8 + p] = 0.25 * c0;
      s_CU[(2 * w + 1) * 8 + p] = 0.25 * c1;
    }
    __syncthreads();
    for (int e = tid; e < 16 * V; e += blockDim.x) {
      const int ell = e >> 3, p = e & 7;
      const int u[4] = {s_lu[4 * ell], s_lu[4 * ell + 1], s_lu[4 * ell + 2], s_lu[4 * ell + 3]};
      double q0 = 0.0, q1 = 0.0, q2 = 0.0;
      if (cp.ke != 0.0) {
        const double *R = s_R + 16 * lk[ell];
        const double g1 = s_G[p * pitch + u[1]], g2 = s_G[p * pitch + u[2]], g3 = s_G[p * pitch + u[3]];
        q0 = cp.ke * (R[4] * g1 + R[8] * g2 + R[12] * g3);
        q1 = cp.ke * (R[9] * g2 + R[13] * g3);
        q2 = cp.ke * (R[14] * g3);
      }
      s_T[u[0] * 8 + p] = q0;
      s_T[u[1] * 8 + p] = q1;
      s_T[u[2] * 8 + p] = q2;
      s_T[u[3] * 8 + p] = 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 8 * n; e += blockDim.x) {
      const int m = e >> 3, p = e & 7, w = m >> 3, j = m & 7;
      s_T[e] += Tn.b[j] * s_CU[(2 * w) * 8 + p] + Tn.b[8 + j] * s_CU[(2 * w + 1) * 8 + p];
    }
    __syncthreads();
    for (int m = part; m < n; m += 32) {
      const double g0 = s_G[p0 * pitch + m], g1 = s_G[(p0 + 1) * pitch + m];
      const double2 t = *reinterpret_cast<const double2 *>(s_T + m * 8 + q0);
      sd00 += g0 * t.x;
      sd01 += g0 * t.y;
      sd10 += g1 * t.x;
      sd11 += g1 * t.y;
    }
  }
  for (int off = 16; off > 0; off >>= 1) {
    sd00 += __shfl_xor(sd00, off, 64);
    sd01 += __shfl_xor(sd01, off, 64);
    sd10 += __shfl_xor(sd10, off, 64);
    sd11 += __shfl_xor(sd11, off, 64);
  }
  __syncthreads();
  double *o = out + static_cast<size_t>(c) * GGF_SENS_STRIDE_DEV;
  if (part == 0) {
    // sum_z (G_z T_z)[p][q] is S_d[q][p]
    o[(2 + q0) * 10 + 2 + p0] = sd00;
    o[(2 + q0 + 1) * 10 + 2 + p0] = sd01;
    o[(2 + q0) * 10 + 2 + p0 + 1] = sd10;
    o[(2 + q0 + 1) * 10 + 2 + p0 + 1] = sd11;
  }
  sens_write_rest(o, s_Sa, s_Sb, s_SN);
}

// ---- Gamma_A sensitivities with K > 1 (L <= 8): per pair (a, b), with M_ab^-1 formed explicitly ----

// M_ab^-1 = G + G_S Y_ab G_S^T of every chain for one ordered pair pr (complex, n x n at
// c * nmax^2 of Gab); chains with K^2 <= pr get G.  s_A: G[:, S] staged per chain.
template <typename T>
__global__ __launch_bounds__(256) void k_form_pair(LaunchCtx lc, int pr, double2 *Gab, int nmax) {
  __shared__ double2 s_Y[16][64];
  __shared__ double2 s_om[16];
  __shared__ int s_S[16][8];
  __shared__ int s_s[16];
  __shared__ double s_A[512 * 8];
  extern __shared__ double2 s_work[];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  pair_setup<T>(lc, c, ch, Tn, G, lk, s_Y, s_om, nullptr, s_S, s_s, s_work);
  const bool has = pr < ch.K * ch.K;
  const int s = has ? s_s[pr] : 0;
  for (int e = threadIdx.x; e < n * s; e += blockDim.x) {
    const int r = e / s, q = e - r * s;
    s_A[r * 8 + q] = static_cast<double>(G[static_cast<size_t>(r) * n + s_S[pr][q]]);
  }
  __syncthreads();
  double2 *out = Gab + static_cast<size_t>(c) * nmax * nmax;
  for (int r = threadIdx.x >> 5; r < n; r += blockDim.x >> 5) {
    double2 ay[8];   // (G_S Y)[r][q], zero for q >= s (fixed trip counts keep it in registers)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double2 v = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < s && q < s) v = cadd(v, cscale(s_Y[pr][p * 8 + q], s_A[r * 8 + p]));
      ay[q] = v;
    }
    for (int col = threadIdx.x & 31; col < n; col += 32) {
      double2 v = make_double2(static_cast<double>(G[static_cast<size_t>(r) * n + col]), 0.0);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < s) v = cadd(v, cscale(ay[q], s_A[col * 8 + q]));
      out[static_cast<size_t>(r) * n + col] = v;
    }
  }
}

// coef * Wc, Wc = (1/4) [[-i, 1], [-1, -i]]: the complex coefficient block of Gamma_out[2x+a][2y+b]
__device__ inline void coef_block_c(double2 coef, double2 o[4]) {
  o[0] = make_double2(0.25 * coef.y, -0.25 * coef.x);
  o[1] = cscale(coef, 0.25);
  o[2] = cscale(coef, -0.25);
  o[3] = o[0];
}

__device__ inline void h_term_c(const EnergyCp &cp, const int8_t *lk, int L, int group, int x, int term, int &w,
                                int &y, double2 o[4]) {
  if (term == 0) {
    const int sgn = (((x % L) + x / L) & 1) ? -1 : 1;
    w = y = x;
    coef_block_c(make_double2(cp.mu + sgn * cp.m, 0.0), o);
    return;
  }
  const int mu = (term - 1) >> 1;
  const int xn = mu == 0 ? ggf_shift(x, L, 1, 0) : ggf_shift(x, L, 0, 1);
  const double2 D = link_phase(lk[2 * x + mu], group);
  const double te = (mu == 0 && ((x / L) & 1)) ? -cp.t : cp.t;
  if ((term & 1) == 1) {
    w = x;
    y = xn;
    coef_block_c(make_double2(-te * D.y, te * D.x), o);
  } else {
    w = xn;
    y = x;
    coef_block_c(make_double2(-te * D.y, -te * D.x), o);
  }
}

// Pair weights of one chain from its energy row: s_wt[0] = om_ab / S = lambda_a^* lambda_b rho_ab / S
// (lambda_a^* lambda_b = w / ov), s_wt[1] = om_ab / S (h_ab - E), E = sum_p lambda^* lambda (rho h / S)_p.
__device__ inline void pair_weights(const TensorDev &Tn, const double *row, int K, int pr, double2 *s_wt) {
  const int a = pr / K, b = pr % K;
  double2 E = make_double2(0.0, 0.0);
  for (int p = 0; p < K * K; ++p) {
    const int pa = p / K, pb = p % K;
    const double2 ll = cdiv(Tn.w[pa][pb], Tn.ov[pa][pb]);
    E = cadd(E, cmul(ll, make_double2(row[3 + 4 * p], row[4 + 4 * p])));
  }
  const double2 rho = make_double2(row[1 + 4 * pr], row[2 + 4 * pr]);
  const double2 rh = make_double2(row[3 + 4 * pr], row[4 + 4 * pr]);
  const double2 om = cmul(cdiv(Tn.w[a][b], Tn.ov[a][b]), rho);
  s_wt[0] = om;
  s_wt[1] = cmul(om, csub(cdiv(rh, rho), E));
}

// M_ab^-1 stored as a complex n x n matrix: entry (r, col), and t_a = sum_j M_ab^-1[r][8w + j] b[a][j].
struct PairInvDense {
  const double2 *Gc;
  int n;
  const double *b;
  __device__ double2 operator()(int r, int col) const { return Gc[static_cast<size_t>(r) * n + col]; }
  __device__ void bcols(int r, int w, double2 &t0, double2 &t1) const {
    const double2 *grow = Gc + static_cast<size_t>(r) * n + 8 * w;
    t0 = t1 = make_double2(0.0, 0.0);
    for (int j = 0; j < 8; ++j) {
      t0 = cadd(t0, cscale(grow[j], b[j]));
      t1 = cadd(t1, cscale(grow[j], b[8 + j]));
    }
  }
};

// M_ab^-1 = G + AY A^T as the rank <= 8 correction of G: AY = G_S Y_ab (n x 8 complex), A = G[:, S]
// (n x 8) and Ab[2w + a][q] = sum_j b[a][j] A[8w + j][q], the columns q >= s zero.
template <typename T>
struct PairInvRank {
  const T *G;
  int n;
  const double *b;
  const double2 *AY;
  const double *A, *Ab;
  __device__ double2 operator()(int r, int col) const {
    double2 v = make_double2(static_cast<double>(G[static_cast<size_t>(r) * n + col]), 0.0);
    const double2 *ay = AY + static_cast<size_t>(r) * 8;
    const double *ac = A + static_cast<size_t>(col) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) v = cadd(v, cscale(ay[q], ac[q]));
    return v;
  }
  __device__ void bcols(int r, int w, double2 &t0, double2 &t1) const {
    const T *grow = G + static_cast<size_t>(r) * n + 8 * w;
    double x0 = 0.0, x1 = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double g = static_cast<double>(grow[j]);
      x0 += g * b[j];
      x1 += g * b[8 + j];
    }
    t0 = make_double2(x0, 0.0);
    t1 = make_double2(x1, 0.0);
    const double2 *ay = AY + static_cast<size_t>(r) * 8;
    const double *ab = Ab + static_cast<size_t>(2 * w) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      t0 = cadd(t0, cscale(ay[q], ab[q]));
      t1 = cadd(t1, cscale(ay[q], ab[8 + q]));
    }
  }
};

// Per-site part of one pair's sensitivities, the K = 1 computation of sens_sites with complex
// blocks and M_ab^-1 read through mi: a-block, b-block and S_N (LDS sums, zeroed by the caller;
// the first wave only, as in sens_sites).
template <typename MI>
__device__ inline void pair_sites(const EnergyCp &cp, const int8_t *lk, int L, int group, const MI &mi, double2 *s_Sa,
                                  double2 *s_Sb, double2 *s_SN) {
  if (threadIdx.x >= 64) return;
  for (int x = threadIdx.x; x < L * L; x += 64) {
    double2 o4[4];
    int w, y;
    h_term_c(cp, lk, L, group, x, 0, w, y, o4);
    for (int aa = 0; aa < 2; ++aa)
      for (int bb = 0; bb < 2; ++bb) {
        atomicAdd(&s_Sa[bb * 2 + aa].x, o4[aa * 2 + bb].x);
        atomicAdd(&s_Sa[bb * 2 + aa].y, o4[aa * 2 + bb].y);
      }
    double2 sb[16];
    for (int q = 0; q < 16; ++q) sb[q] = make_double2(0.0, 0.0);
    for (int nb = 0; nb < 5; ++nb) {
      int yy = x;
      if (nb == 1) yy = ggf_shift(x, L, 1, 0);
      if (nb == 2) yy = ggf_shift(x, L, 0, 1);
      if (nb == 3) yy = ggf_shift(x, L, -1, 0);
      if (nb == 4) yy = ggf_shift(x, L, 0, -1);
      if ((nb == 3 && yy == ggf_shift(x, L, 1, 0)) || (nb == 4 && yy == ggf_shift(x, L, 0, 1))) continue;
      double2 orow[4], ocol[4];
      for (int q = 0; q < 4; ++q) orow[q] = ocol[q] = make_double2(0.0, 0.0);
      const int owners[2] = {x, yy};
      for (int oi = 0; oi < (nb == 0 ? 1 : 2); ++oi)
        for (int term = 0; term < 5; ++term) {
          if ((nb == 0) != (term == 0)) continue;
          int w2, y2;
          double2 ot[4];
          h_term_c(cp, lk, L, group, owners[oi], term, w2, y2, ot);
          if (w2 == x && y2 == yy)
            for (int q = 0; q < 4; ++q) orow[q] = cadd(orow[q], ot[q]);
          if (w2 == yy && y2 == x)
            for (int q = 0; q < 4; ++q) ocol[q] = cadd(ocol[q], ot[q]);
        }
      if (nb == 0)
        for (int q = 0; q < 4; ++q) ocol[q] = orow[q];
      for (int i = 0; i < 8; ++i) {
        double2 t0, t1;
        mi.bcols(8 * x + i, yy, t0, t1);
        for (int aa = 0; aa < 2; ++aa) {
          sb[aa * 8 + i] = cadd(sb[aa * 8 + i], cadd(cmul(orow[aa * 2 + 0], t0), cmul(orow[aa * 2 + 1], t1)));
          sb[aa * 8 + i] = csub(sb[aa * 8 + i], cadd(cmul(ocol[0 * 2 + aa], t0), cmul(ocol[1 * 2 + aa], t1)));
        }
      }
    }
    for (int q = 0; q < 16; ++q) {
      atomicAdd(&s_Sb[q].x, sb[q].x);
      atomicAdd(&s_Sb[q].y, sb[q].y);
    }
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        const double2 g = mi(8 * x + i, 8 * x + j);
        atomicAdd(&s_SN[i * 8 + j].x, 0.5 * g.x);
        atomicAdd(&s_SN[i * 8 + j].y, 0.5 * g.y);
      }
  }
}

// Writes (pr == 0) or adds one pair's weighted a-block, b-block and S_N (thread tid < 100 its share):
// S_e += Re (om/S) S_e^ab, S_N += Re (om/S) S_N^ab, and the zero entries.
__device__ inline void pair_write_rest(double *o, bool first, double2 w0, const double2 *s_Sa, const double2 *s_Sb,
                                       const double2 *s_SN) {
  const int tid = threadIdx.x;
  auto put = [&](int idx, double v) { o[idx] = first ? v : o[idx] + v; };
  if (tid < 64) put(100 + (2 + (tid >> 3)) * 10 + 2 + (tid & 7), cmul(w0, s_SN[tid]).x);
  if (tid < 16) {
    const int al = tid >> 3, i = tid & 7;
    put((2 + i) * 10 + al, cmul(w0, s_Sb[tid]).x);
  }
  if (tid < 4) put((tid >> 1) * 10 + (tid & 1), cmul(w0, s_Sa[tid]).x);
  if (tid < 20) {
    const int al = tid / 10, j = tid % 10;
    if (j >= 2) put(al * 10 + j, 0.0);
  }
  if (tid < 100) {
    const int i = tid / 10, j = tid % 10;
    if (i < 2 || j < 2) put(100 + tid, 0.0);
  }
}

// One pair's contribution to the K > 1 sensitivities of a chain (the K = 1 computation of
// k_sens with the complex M_ab^-1 of Gab and the pair's electric slopes), weighted by the
// pair's om / S and combined with h_ab and E from the chain's energy row:
//   S_e += Re (om/S) [S_e^ab + (h_ab - E) S_N^ab],   S_N += Re (om/S) S_N^ab.
// pr == 0 writes the row, later pairs add to it.  L <= 8; launched with 512 threads.
__global__ __launch_bounds__(512, 2) void k_sens_pair(LaunchCtx lc, EnergyCp cp, int pr, const double2 *Gab, int nmax,
                                                   const double *erows, double *out) {
  // dynamic LDS: T_z[m][p] (n x 8, U_z[2w + a][i] at its start), CU[2w + a][p] (2V x 8), the block
  // coefficients of each row site (5 V, complex), their column sites (int16) and the links' Majoranas (int16)
  extern __shared__ double2 s_dyn2[];
  double2 *s_T = s_dyn2;
  double2 *s_U = s_T;
  double2 *s_CU = s_T + 8 * nmax;
  double2 *s_cc = s_CU + 2 * nmax;
  int16_t *s_cy = reinterpret_cast<int16_t *>(s_cc + 5 * (nmax / 8));
  int16_t *s_lu = s_cy + 5 * (nmax / 8);
  __shared__ double2 s_sl[128][6];        // electric slopes of the pair per link
  __shared__ double2 s_Sa[4], s_Sb[16], s_SN[64];
  __shared__ double2 s_wt[2];             // om/S, om/S (h - E)
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, group = ch.group, K = ch.K;
  const int8_t *lk = lc.links + ch.link_off;
  const int tid = threadIdx.x;
  double *o = out + static_cast<size_t>(c) * GGF_SENS_STRIDE_DEV;
  if (pr >= K * K) return;
  const int a = pr / K, b = pr % K;
  const double2 *Gc = Gab + static_cast<size_t>(c) * nmax * nmax;
  if (tid == 0) pair_weights(Tn, erows + static_cast<size_t>(c) * GGF_ENERGY_STRIDE_DEV, K, pr, s_wt);
  if (tid < 4) s_Sa[tid] = make_double2(0.0, 0.0);
  if (tid < 16) s_Sb[tid] = make_double2(0.0, 0.0);
  if (tid < 64) s_SN[tid] = make_double2(0.0, 0.0);
  for (int ell = tid; ell < 2 * V; ell += blockDim.x) {
    // slope of the pair's X along e_ij - e_ji: R[j][i], R = O eq_ab O^T of this link
    const double2 *eq = Tn.eq0;
    for (int l = 0; l < Tn.nl[a][b]; ++l)
      if (Tn.lk[a][b][l] == ell) eq = Tn.eq[a][b][l];
    int k = 0;
    for (int i = 0; i < 4; ++i) {
      for (int j = i + 1; j < 4; ++j) {
        double2 row[4];
        rotate_dg_row(eq, lk[ell], group, j, row);   // row j of O eq O^T
        s_sl[ell][k++] = row[i];
      }
    }
    int u[4];
    ggf_link_u(ell, L, u);
    for (int q = 0; q < 4; ++q) s_lu[4 * ell + q] = static_cast<int16_t>(u[q]);
  }
  for (int e = tid; e < 5 * V; e += blockDim.x) {
    // row site w: on site, the hops to w + e1 and w + e2 (terms 1, 3 of w), the reverse hops from
    // w - e1 and w - e2 (terms 2, 4 of those sites)
    const int w = e / 5, t = e - 5 * w;
    int owner = w, term = t;
    if (t == 2) term = 3;
    else if (t == 3) { owner = ggf_shift(w, L, -1, 0); term = 2; }
    else if (t == 4) { owner = ggf_shift(w, L, 0, -1); term = 4; }
    int wr, y;
    s_cc[e] = h_coef(cp, lk, L, group, owner, term, wr, y);
    s_cy[e] = static_cast<int16_t>(y);
  }
  __syncthreads();
  pair_sites(cp, lk, L, group, PairInvDense{Gc, n, Tn.b}, s_Sa, s_Sb, s_SN);
  // d-block in two contractions per row stripe z (as k_sens_t, complex):
  //   CU = C U_z^T, T_z = b^T CU + the pair's electric slopes, acc(p, q) += sum_m M_ab^-1[8z + p][m] T_z[m][q]
  const int part = tid & 31, blk = tid >> 5;
  const int p0 = 2 * (blk >> 2), q0 = 2 * (blk & 3);
  double2 sd[4];
  for (int q = 0; q < 4; ++q) sd[q] = make_double2(0.0, 0.0);
  for (int z = 0; z < V; ++z) {
    __syncthreads();
    // U_z[2w + a][i]: 16 V <= 1024 items, two per thread with their loads issued together
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + 512 * k;
      if (e < 16 * V) {
        const int i = e & 7, col = e >> 3, w = col >> 1, al = col & 1;
        const double2 *grow = Gc + static_cast<size_t>(8 * z + i) * n + 8 * w;
        double2 v = make_double2(0.0, 0.0);
        for (int jj = 0; jj < 8; ++jj) v = cadd(v, cscale(grow[jj], Tn.b[al * 8 + jj]));
        s_U[e] = v;
      }
    }
    __syncthreads();
    for (int e = tid; e < 8 * V; e += blockDim.x) {
      const int w = e >> 3, p = e & 7;
      double2 c0 = make_double2(0.0, 0.0), c1 = make_double2(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        double2 o4[4];
        coef_block_c(s_cc[5 * w + t], o4);
        const int y = s_cy[5 * w + t];
        const double2 u0 = s_U[(2 * y) * 8 + p], u1 = s_U[(2 * y + 1) * 8 + p];
        c0 = cadd(c0, cadd(cmul(o4[0], u0), cmul(o4[1], u1)));
        c1 = cadd(c1, cadd(cmul(o4[2], u0), cmul(o4[3], u1)));
      }
      s_CU[(2 * w) * 8 + p] = c0;
      s_CU[(2 * w + 1) * 8 + p] = c1;
    }
    __syncthreads();
    for (int e = tid; e < 16 * V; e += blockDim.x) {
      const int ell = e >> 3, p = e & 7;
      const int u[4] = {s_lu[4 * ell], s_lu[4 * ell + 1], s_lu[4 * ell + 2], s_lu[4 * ell + 3]};
      double2 q0v = make_double2(0.0, 0.0), q1v = q0v, q2v = q0v;
      if (cp.ke != 0.0) {
        const double2 *grow = Gc + static_cast<size_t>(8 * z + p) * n;
        const double2 g1 = grow[u[1]], g2 = grow[u[2]], g3 = grow[u[3]];
        // s_sl[ell]: R[1][0], R[2][0], R[3][0], R[2][1], R[3][1], R[3][2]
        q0v = cscale(cadd(cadd(cmul(s_sl[ell][0], g1), cmul(s_sl[ell][1], g2)), cmul(s_sl[ell][2], g3)), cp.ke);
        q1v = cscale(cadd(cmul(s_sl[ell][3], g2), cmul(s_sl[ell][4], g3)), cp.ke);
        q2v = cscale(cmul(s_sl[ell][5], g3), cp.ke);
      }
      s_T[u[0] * 8 + p] = q0v;
      s_T[u[1] * 8 + p] = q1v;
      s_T[u[2] * 8 + p] = q2v;
      s_T[u[3] * 8 + p] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < 8 * n; e += blockDim.x) {
      const int m = e >> 3, p = e & 7, w = m >> 3, jj = m & 7;
      s_T[e] = cadd(s_T[e], cadd(cscale(s_CU[(2 * w) * 8 + p], Tn.b[jj]), cscale(s_CU[(2 * w + 1) * 8 + p], Tn.b[8 + jj])));
    }
    __syncthreads();
    const double2 *r0 = Gc + static_cast<size_t>(8 * z + p0) * n, *r1 = r0 + n;
    for (int m = part; m < n; m += 32) {
      const double2 g0 = r0[m], g1 = r1[m], t0 = s_T[m * 8 + q0], t1 = s_T[m * 8 + q0 + 1];
      sd[0] = cadd(sd[0], cmul(g0, t0));
      sd[1] = cadd(sd[1], cmul(g0, t1));
      sd[2] = cadd(sd[2], cmul(g1, t0));
      sd[3] = cadd(sd[3], cmul(g1, t1));
    }
  }
  for (int off = 16; off > 0; off >>= 1)
    for (int q = 0; q < 4; ++q) {
      sd[q].x += __shfl_xor(sd[q].x, off, 64);
      sd[q].y += __shfl_xor(sd[q].y, off, 64);
    }
  __syncthreads();
  // combine: S_e^ab entries e and S_N^ab entries n: row += Re(om/S e + om/S (h - E) n), S_N += Re(om/S n)
  const double2 w0 = s_wt[0], w1 = s_wt[1];
  const bool first = pr == 0;
  auto put = [&](int idx, double v) { o[idx] = first ? v : o[idx] + v; };
  if (part == 0)
    for (int q = 0; q < 4; ++q) {
      // acc(p, q') is S_d^ab[q'][p]; S_N^ab[2 + q'][2 + p] = s_SN[q' * 8 + p]
      const int pp = p0 + (q >> 1), qq = q0 + (q & 1);
      put((2 + qq) * 10 + 2 + pp, cmul(w0, sd[q]).x + cmul(w1, s_SN[qq * 8 + pp]).x);
    }
  pair_write_rest(o, first, w0, s_Sa, s_Sb, s_SN);
}

// ---- Gamma_A sensitivities with K > 1 at any L <= 32: M_ab^-1 = G + AY A^T applied on the fly ----

// Per chain and ordered pair pr, the factors of the rank <= 8 correction M_ab^-1 - G (PairInvRank):
// A = G[:, S] and AY = A Y_ab at c * nmax * 8, Ab at c * (nmax / 4) * 8; s = 0 (all zero) for the
// pair (0, 0) and for chains with K^2 <= pr.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_tables(LaunchCtx lc, int pr, double2 *AY, double *A, double *Ab,
                                                     int nmax) {
  __shared__ double2 s_Y[16][64];
  __shared__ double2 s_om[16];
  __shared__ int s_S[16][8];
  __shared__ int s_s[16];
  extern __shared__ double2 s_work[];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  pair_setup<T>(lc, c, ch, Tn, G, lk, s_Y, s_om, nullptr, s_S, s_s, s_work);
  const int s = pr < ch.K * ch.K ? s_s[pr] : 0;
  double2 *ay = AY + static_cast<size_t>(c) * nmax * 8;
  double *ag = A + static_cast<size_t>(c) * nmax * 8;
  double *ab = Ab + static_cast<size_t>(c) * (nmax / 4) * 8;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double g[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) g[q] = q < s ? static_cast<double>(G[static_cast<size_t>(r) * n + s_S[pr][q]]) : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double2 v = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < s && q < s) v = cadd(v, cscale(s_Y[pr][p * 8 + q], g[p]));
      ay[static_cast<size_t>(r) * 8 + q] = v;
      ag[static_cast<size_t>(r) * 8 + q] = g[q];
    }
  }
  for (int e = threadIdx.x; e < 2 * n; e += blockDim.x) {
    // Ab[2w + al][q], e = (2w + al) * 8 + q
    const int row = e >> 3, q = e & 7, w = row >> 1, al = row & 1;
    double v = 0.0;
    if (q < s)
      for (int j = 0; j < 8; ++j) v += Tn.b[al * 8 + j] * static_cast<double>(G[static_cast<size_t>(8 * w + j) * n + s_S[pr][q]]);
    ab[e] = v;
  }
}

// The d-block of one pair's contribution to the K > 1 sensitivities, om/S S_d^ab as in k_sens_pair (written
// for pr == 0, else added), with M_ab^-1 = G + AY A^T read through the correction, per row stripe z in chunks
// of lattice rows as in k_sens:
//   hopping part: U_z[i][2w + a] = sum_j M_ab^-1[8z + i][8w + j] b[a][j] of the chunk's sites in LDS;
//   electric part, with R_l the pair's slopes and the expansion of M_ab^-1 = G + AY A^T,
//     sum_l sum_{i<j} R_l[j][i] M[P][u_j] M[Q][u_i] = sum_l sum_{i<j} R_l[j][i] G[P][u_j] G[Q][u_i]
//       + sum_q AY[Q][q] Xa[P][q] + sum_q AY[P][q] Xb[Q][q] + sum_{q,q'} AY[P][q] Z[q][q'] AY[Q][q'],
//     Xa[P][q] = sum R[j][i] G[P][u_j] A[u_i][q], Xb[Q][q] = sum R[j][i] A[u_j][q] G[Q][u_i] (per stripe) and
//     Z[q][q'] = sum R[j][i] A[u_j][q] A[u_i][q'] (once per chain and pair).
// At most kPairSites sites per chunk (R = min(L, kPairSites / L - 1) rows and the row after them).
// Launched with 256 threads: thread (pi, pj) of each of the 4 parts sums the d-block entry (pi, pj).
constexpr int kPairSites = 224;
template <typename T>
__global__ __launch_bounds__(256) void k_sens_pair_rows(LaunchCtx lc, EnergyCp cp, int pr, const double2 *AY,
                                                        const double *A, const double *Ab, int nmax,
                                                        const double *erows, double *out) {
  extern __shared__ double2 s_dyn2[];
  double2 *s_U = s_dyn2;                      // U_z[i][2 ls + a], ls the chunk's site
  __shared__ double2 s_ph[GGF_ZN_MAX];        // link phases exp(2 pi i k / N)
  __shared__ double2 s_Rg[GGF_ZN_MAX][6];     // slopes R[1][0], R[2][0], R[3][0], R[2][1], R[3][1], R[3][2] per link value
  __shared__ double2 s_Rp[2][6];              // the same for the pair's patch links
  __shared__ int s_pl[2];
  __shared__ double2 s_wt[2], s_Z[64];
  __shared__ double2 s_X[4][2][64];           // per part: Xa[P][q], Xb[Q][q] of the stripe
  __shared__ double2 s_red[4][64];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int n = ch.n, L = ch.L, V = L * L, group = ch.group, K = ch.K;
  if (pr >= K * K) return;
  const int a = pr / K, b = pr % K;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const int8_t *lk = lc.links + ch.link_off;
  const double2 *ay = AY + static_cast<size_t>(c) * nmax * 8;
  const double *ag = A + static_cast<size_t>(c) * nmax * 8;
  const PairInvRank<T> mi{G, n, Tn.b, ay, ag, Ab + static_cast<size_t>(c) * (nmax / 4) * 8};
  const int tid = threadIdx.x;
  if (tid == 0) pair_weights(Tn, erows + static_cast<size_t>(c) * GGF_ENERGY_STRIDE_DEV, K, pr, s_wt);
  if (tid < 2) s_pl[tid] = tid < Tn.nl[a][b] ? Tn.lk[a][b][tid] : -1;
  for (int k = tid; k < group; k += blockDim.x) s_ph[k] = link_phase(k, group);
  for (int te = tid; te < 6 * (group + 2); te += blockDim.x) {
    // entry idx of (i, j) = (0,1), (0,2), (0,3), (1,2), (1,3), (2,3): R[j][i], row j of O eq O^T
    const int k = te / 6, idx = te - 6 * k;
    const int i = idx < 3 ? 0 : (idx < 5 ? 1 : 2);
    const int j = idx < 3 ? idx + 1 : (idx < 5 ? idx - 1 : 3);
    double2 row[4];
    if (k < group) {
      rotate_dg_row(Tn.eq0, k, group, j, row);
      s_Rg[k][idx] = row[i];
    } else if (k - group < Tn.nl[a][b]) {
      const int l = k - group;
      rotate_dg_row(Tn.eq[a][b][l], lk[Tn.lk[a][b][l]], group, j, row);
      s_Rp[l][idx] = row[i];
    }
  }
  __syncthreads();
  // a link's slopes: a patch link of the pair (the later entry first), else the unpatched link's
  auto slopes = [&](int ell) -> const double2 * {
    if (ell == s_pl[1]) return s_Rp[1];
    if (ell == s_pl[0]) return s_Rp[0];
    return s_Rg[lk[ell]];
  };
  const int ij = tid & 63, part = tid >> 6;
  const int pi = ij >> 3, pj = ij & 7;
  if (cp.ke != 0.0) {
    // Z[q][q'] with thread (pi, pj) taking q = pi, q' = pj
    double2 zv = make_double2(0.0, 0.0);
    for (int ell = part; ell < 2 * V; ell += 4) {
      int u[4];
      ggf_link_u(ell, L, u);
      const double2 *R = slopes(ell);
      double aq[4], ar[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        aq[k] = ag[static_cast<size_t>(u[k]) * 8 + pi];
        ar[k] = ag[static_cast<size_t>(u[k]) * 8 + pj];
      }
      int k = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j) zv = cadd(zv, cscale(R[k++], aq[j] * ar[i]));
    }
    s_red[part][ij] = zv;
  }
  __syncthreads();
  if (tid < 64)
    s_Z[tid] = cp.ke != 0.0 ? cscale(cadd(cadd(s_red[0][tid], s_red[1][tid]), cadd(s_red[2][tid], s_red[3][tid])), cp.ke)
                            : make_double2(0.0, 0.0);
  const int R = min(L, kPairSites / L - 1);
  // index of site s among the chunk's sites (rows r0 .. r0 + nr, the last taken mod L)
  auto local = [&](int s_, int r0) { return (((s_ / L) - r0 + L) % L) * L + s_ % L; };
  double2 sd = make_double2(0.0, 0.0);
  for (int z = 0; z < V; ++z) {
    double2 acc = make_double2(0.0, 0.0);
    for (int r0 = 0; r0 < L; r0 += R) {
      const int nr = min(R, L - r0);
      const int ns = (nr + 1) * L;
      __syncthreads();                        // readers of the previous chunk's U_z (and s_X) are done
      for (int e = tid; e < 8 * ns; e += blockDim.x) {
        const int i = e / ns, ls = e - i * ns;
        const int w = ((r0 + ls / L) % L) * L + ls % L;
        double2 t0, t1;
        mi.bcols(8 * z + i, w, t0, t1);
        s_U[i * 2 * ns + 2 * ls] = t0;
        s_U[i * 2 * ns + 2 * ls + 1] = t1;
      }
      __syncthreads();
      for (int lx = part; lx < nr * L; lx += 4) {
        const int x = (r0 + lx / L) * L + lx % L;
#pragma unroll
        for (int term = 0; term < 5; ++term) {
          const double2 D = term == 0 ? make_double2(1.0, 0.0) : s_ph[lk[2 * x + ((term - 1) >> 1)]];
          int w, y;
          double2 o4[4];
          coef_block_c(h_coef_d(cp, L, x, term, D, w, y), o4);
          const int lw = local(w, r0), ly = local(y, r0);
          const double2 ui0 = s_U[pi * 2 * ns + 2 * lw], ui1 = s_U[pi * 2 * ns + 2 * lw + 1];
          const double2 uj0 = s_U[pj * 2 * ns + 2 * ly], uj1 = s_U[pj * 2 * ns + 2 * ly + 1];
          acc = cadd(acc, cmul(ui0, cadd(cmul(o4[0], uj0), cmul(o4[1], uj1))));
          acc = cadd(acc, cmul(ui1, cadd(cmul(o4[2], uj0), cmul(o4[3], uj1))));
        }
      }
    }
    if (cp.ke != 0.0) {
      // P = 8z + pj (u_j), Q = 8z + pi (u_i)
      const T *gp = G + static_cast<size_t>(8 * z + pj) * n, *gq = G + static_cast<size_t>(8 * z + pi) * n;
      double2 ee = make_double2(0.0, 0.0), xa = ee, xb = ee;
      for (int ell = part; ell < 2 * V; ell += 4) {
        int u[4];
        ggf_link_u(ell, L, u);
        const double2 *Rl = slopes(ell);
        double vp[4], vq[4], api[4], apj[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          vp[k] = static_cast<double>(gp[u[k]]);
          vq[k] = static_cast<double>(gq[u[k]]);
          api[k] = ag[static_cast<size_t>(u[k]) * 8 + pi];
          apj[k] = ag[static_cast<size_t>(u[k]) * 8 + pj];
        }
        int k = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = i + 1; j < 4; ++j) {
            const double2 r = Rl[k++];
            ee = cadd(ee, cscale(r, vp[j] * vq[i]));
            xa = cadd(xa, cscale(r, vp[j] * api[i]));   // Xa[pj][pi]
            xb = cadd(xb, cscale(r, apj[j] * vq[i]));   // Xb[pi][pj]
          }
      }
      s_X[part][0][pj * 8 + pi] = cscale(xa, cp.ke);
      s_X[part][1][pi * 8 + pj] = cscale(xb, cp.ke);
      acc = cadd(acc, cscale(ee, cp.ke));
      __syncthreads();
      const double2 *ayq = ay + static_cast<size_t>(8 * z + pi) * 8, *ayp = ay + static_cast<size_t>(8 * z + pj) * 8;
      double2 corr = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        corr = cadd(corr, cmul(ayq[q], s_X[part][0][pj * 8 + q]));
        corr = cadd(corr, cmul(ayp[q], s_X[part][1][pi * 8 + q]));
      }
      if (part == 0)
        for (int q = 0; q < 8; ++q) {
          double2 zq = make_double2(0.0, 0.0);
#pragma unroll
          for (int q2 = 0; q2 < 8; ++q2) zq = cadd(zq, cmul(s_Z[q * 8 + q2], ayq[q2]));
          corr = cadd(corr, cmul(ayp[q], zq));
        }
      acc = cadd(acc, corr);
    }
    sd = cadd(sd, acc);
  }
  __syncthreads();
  s_red[part][ij] = sd;
  __syncthreads();
  double *o = out + static_cast<size_t>(c) * GGF_SENS_STRIDE_DEV;
  if (tid < 64) {
    // thread (pi, pj) summed (U C U^T)[pi][pj] + electric part: S_d^ab[pj][pi]
    const double2 v = cadd(cadd(s_red[0][tid], s_red[1][tid]), cadd(s_red[2][tid], s_red[3][tid]));
    const int idx = (2 + pj) * 10 + 2 + pi;
    const double add = cmul(s_wt[0], v).x;
    o[idx] = pr == 0 ? add : o[idx] + add;
  }
}

// The rest of one pair's contribution after k_sens_pair_rows: a-block, b-block and S_N with M_ab^-1 read
// through the correction, and the S_N part of the d-block, om/S (h_ab - E) S_N^ab (added).  A kernel of
// its own so that the per-site registers do not bound the occupancy of the stripe contraction.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_sites(LaunchCtx lc, EnergyCp cp, int pr, const double2 *AY,
                                                    const double *A, const double *Ab, int nmax, const double *erows,
                                                    double *out) {
  __shared__ double2 s_Sa[4], s_Sb[16], s_SN[64], s_wt[2];
  const int c = blockIdx.x;
  const ChainDev ch = lc.chains[c];
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const int K = ch.K, tid = threadIdx.x;
  if (pr >= K * K) return;
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  const PairInvRank<T> mi{G, ch.n, Tn.b, AY + static_cast<size_t>(c) * nmax * 8, A + static_cast<size_t>(c) * nmax * 8,
                          Ab + static_cast<size_t>(c) * (nmax / 4) * 8};
  if (tid == 0) pair_weights(Tn, erows + static_cast<size_t>(c) * GGF_ENERGY_STRIDE_DEV, K, pr, s_wt);
  if (tid < 4) s_Sa[tid] = make_double2(0.0, 0.0);
  if (tid < 16) s_Sb[tid] = make_double2(0.0, 0.0);
  if (tid < 64) s_SN[tid] = make_double2(0.0, 0.0);
  __syncthreads();
  pair_sites(cp, lc.links + ch.link_off, ch.L, ch.group, mi, s_Sa, s_Sb, s_SN);
  __syncthreads();
  double *o = out + static_cast<size_t>(c) * GGF_SENS_STRIDE_DEV;
  if (tid < 64) {
    const int pi = tid >> 3, pj = tid & 7;
    o[(2 + pj) * 10 + 2 + pi] += cmul(s_wt[1], s_SN[pj * 8 + pi]).x;
  }
  pair_write_rest(o, pr == 0, s_wt[0], s_Sa, s_Sb, s_SN);
}
}  // namespace

static size_t pair_lds(int kmax) {
  const int np = kmax * (kmax + 1) / 2 - 1;
  return np > 0 ? static_cast<size_t>(np) * kPairLd * kPairLd * sizeof(double2) : 0;
}

void ggf_launch_ratio(const LaunchCtx &lc, int ell, int parity, int kmax, int t, int wp) {
  // pair workspaces, then for delayed updates H (nIm x 4F), G_AI (4F x nIm) and (nIm + 4) x 4F
  // scratch, nIm the largest index set of the context (4 without pairs)
  const bool pairs = kmax > 1;
  const int nIm = pairs ? lc.nidx : 4;
  const size_t lds = pair_lds(kmax) + (lc.dly > 0 ? static_cast<size_t>(3 * nIm + 4) * 4 * lc.dly * sizeof(double) : 0);
  const void *fn = lc.precision == 64
                       ? (pairs ? reinterpret_cast<const void *>(&k_ratio<double, true>)
                                : reinterpret_cast<const void *>(&k_ratio<double, false>))
                       : (pairs ? reinterpret_cast<const void *>(&k_ratio<float, true>)
                                : reinterpret_cast<const void *>(&k_ratio<float, false>));
  // 9 pair workspaces (K = 4, 36 KB) with a 32-step window exceed the default 64 KB of
  // dynamic LDS: raise the limit to what this launch needs (the launch reports an error
  // if the device cannot provide it)
  static size_t lds_set[4] = {64 * 1024, 64 * 1024, 64 * 1024, 64 * 1024};
  const int ti = (lc.precision == 64 ? 0 : 2) + (pairs ? 1 : 0);
  if (lds > lds_set[ti]) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) == hipSuccess)
      lds_set[ti] = lds;
    else
      (void)hipGetLastError();
  }
  if (lc.precision == 64) {
    if (pairs)
      hipLaunchKernelGGL((k_ratio<double, true>), dim3(lc.n_chains), dim3(kRatioThreads), lds, lc.stream, lc, ell,
                         parity, t, wp);
    else
      hipLaunchKernelGGL((k_ratio<double, false>), dim3(lc.n_chains), dim3(kRatioThreads), lds, lc.stream, lc, ell,
                         parity, t, wp);
  } else {
    if (pairs)
      hipLaunchKernelGGL((k_ratio<float, true>), dim3(lc.n_chains), dim3(kRatioThreads), lds, lc.stream, lc, ell,
                         parity, t, wp);
    else
      hipLaunchKernelGGL((k_ratio<float, false>), dim3(lc.n_chains), dim3(kRatioThreads), lds, lc.stream, lc, ell,
                         parity, t, wp);
  }
}

void ggf_launch_update(const LaunchCtx &lc, int parity, int grid, int tiles, int nt) {
  grid = ((grid + 7) / 8) * 8;   // the XCD mapping needs a multiple of 8 workgroups
  if (lc.precision == 64) {
    if (nt) hipLaunchKernelGGL((k_update<double, true>), dim3(grid), dim3(256), 0, lc.stream, lc, parity, tiles);
    else hipLaunchKernelGGL((k_update<double, false>), dim3(grid), dim3(256), 0, lc.stream, lc, parity, tiles);
  } else {
    if (nt) hipLaunchKernelGGL((k_update<float, true>), dim3(grid), dim3(256), 0, lc.stream, lc, parity, tiles);
    else hipLaunchKernelGGL((k_update<float, false>), dim3(grid), dim3(256), 0, lc.stream, lc, parity, tiles);
  }
}

void ggf_launch_end_sweep(const LaunchCtx &lc) {
  hipLaunchKernelGGL(k_end_sweep, dim3((lc.n_chains + 255) / 256), dim3(256), 0, lc.stream, lc);
}

void ggf_launch_hot_start(const LaunchCtx &lc, int max_links) {
  hipLaunchKernelGGL(k_hot_start, dim3((max_links + 255) / 256, lc.n_chains), dim3(256), 0, lc.stream, lc,
                     max_links);
}

void ggf_launch_sfac(const LaunchCtx &lc, const int *list, int count, int kmax) {
  const size_t lds = pair_lds(kmax);
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_sfac<double>, dim3(count), dim3(64), lds, lc.stream, lc, list, count);
  else
    hipLaunchKernelGGL(k_sfac<float>, dim3(count), dim3(64), lds, lc.stream, lc, list, count);
}

void ggf_launch_energy(const LaunchCtx &lc, const EnergyCp &cp, double *out, int kmax) {
  const size_t lds = kmax > 1 ? 4 * (kPairLd * kPairLd + 64) * sizeof(double2) : 0;
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_energy<double>, dim3(lc.n_chains), dim3(256), lds, lc.stream, lc, cp, out);
  else
    hipLaunchKernelGGL(k_energy<float>, dim3(lc.n_chains), dim3(256), lds, lc.stream, lc, cp, out);
}

void ggf_launch_bond_rows(const LaunchCtx &lc, const EnergyCp &cp, double *out) {
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_bond_rows<double>, dim3(lc.n_chains), dim3(256), 0, lc.stream, lc, cp, out);
  else
    hipLaunchKernelGGL(k_bond_rows<float>, dim3(lc.n_chains), dim3(256), 0, lc.stream, lc, cp, out);
}

void ggf_launch_sens(const LaunchCtx &lc, const EnergyCp &cp, double *out, int max_sites, int max_group) {
  const dim3 grid(lc.n_chains), block(256);
  if (max_sites <= 100) {
    const dim3 block512(512);
    // two-stage stripe contraction: stripe, T_z (U_z inside), CU and the tables in LDS (80.8 KB at V = 64)
    const size_t lds = (static_cast<size_t>(144) * max_sites + 16 + 16 * max_group) * sizeof(double) +
                       static_cast<size_t>(5) * max_sites * sizeof(double2) + static_cast<size_t>(13) * max_sites * 2;
    if (lc.precision == 64)
      hipLaunchKernelGGL(k_sens_t<double>, grid, block512, lds, lc.stream, lc, cp, out, max_sites, max_group);
    else
      hipLaunchKernelGGL(k_sens_t<float>, grid, block512, lds, lc.stream, lc, cp, out, max_sites, max_group);
    return;
  }
  // one-stage kernel: U_z of a chunk of lattice rows in LDS (kSensSites sites, 56 KB)
  const size_t lds_u = static_cast<size_t>(16) * kSensSites * sizeof(double);
  if (lc.precision == 64) hipLaunchKernelGGL(k_sens<double>, grid, block, lds_u, lc.stream, lc, cp, out, max_sites);
  else hipLaunchKernelGGL(k_sens<float>, grid, block, lds_u, lc.stream, lc, cp, out, max_sites);
}

size_t ggf_sens_pairs_scratch(int n_chains, int nmax) {
  const size_t per = nmax <= 512 ? static_cast<size_t>(nmax) * nmax * sizeof(double2)
                                 : static_cast<size_t>(nmax) * 8 * (sizeof(double2) + sizeof(double)) +
                                       static_cast<size_t>(nmax / 4) * 8 * sizeof(double);
  return static_cast<size_t>(n_chains) * per;
}

void ggf_launch_sens_pairs(const LaunchCtx &lc, const EnergyCp &cp, void *scratch, int nmax, const double *erows,
                           double *out, int kmax) {
  const size_t lds = kmax > 1 ? 4 * (kPairLd * kPairLd + 64) * sizeof(double2) : 0;
  const dim3 grid(lc.n_chains);
  const bool f64 = lc.precision == 64;
  if (nmax > 512) {
    // per pair: the correction tables, the row-chunked contraction (U_z of kPairSites sites, 56 KB), the
    // per-site part
    double2 *AY = static_cast<double2 *>(scratch);
    double *A = reinterpret_cast<double *>(AY + static_cast<size_t>(lc.n_chains) * nmax * 8);
    double *Ab = A + static_cast<size_t>(lc.n_chains) * nmax * 8;
    const size_t lds_u = static_cast<size_t>(16) * kPairSites * sizeof(double2);
    for (int pr = 0; pr < kmax * kmax; ++pr) {
      if (f64) {
        hipLaunchKernelGGL(k_pair_tables<double>, grid, dim3(256), lds, lc.stream, lc, pr, AY, A, Ab, nmax);
        hipLaunchKernelGGL(k_sens_pair_rows<double>, grid, dim3(256), lds_u, lc.stream, lc, cp, pr, AY, A, Ab, nmax,
                           erows, out);
        hipLaunchKernelGGL(k_pair_sites<double>, grid, dim3(256), 0, lc.stream, lc, cp, pr, AY, A, Ab, nmax, erows,
                           out);
      } else {
        hipLaunchKernelGGL(k_pair_tables<float>, grid, dim3(256), lds, lc.stream, lc, pr, AY, A, Ab, nmax);
        hipLaunchKernelGGL(k_sens_pair_rows<float>, grid, dim3(256), lds_u, lc.stream, lc, cp, pr, AY, A, Ab, nmax,
                           erows, out);
        hipLaunchKernelGGL(k_pair_sites<float>, grid, dim3(256), 0, lc.stream, lc, cp, pr, AY, A, Ab, nmax, erows,
                           out);
      }
    }
    return;
  }
  double2 *gab = static_cast<double2 *>(scratch);
  // k_sens_pair: T_z (8 n), CU (2 n), coefficients (5 V) complex; column sites (5 V), Majoranas (n) int16
  const size_t lds_s = (static_cast<size_t>(10) * nmax + 5 * (nmax / 8)) * sizeof(double2) +
                       (static_cast<size_t>(5) * (nmax / 8) + nmax) * sizeof(int16_t);
  for (int pr = 0; pr < kmax * kmax; ++pr) {
    if (f64)
      hipLaunchKernelGGL(k_form_pair<double>, grid, dim3(256), lds, lc.stream, lc, pr, gab, nmax);
    else
      hipLaunchKernelGGL(k_form_pair<float>, grid, dim3(256), lds, lc.stream, lc, pr, gab, nmax);
    hipLaunchKernelGGL(k_sens_pair, grid, dim3(512), lds_s, lc.stream, lc, cp, pr, gab, nmax, erows, out);
  }
}

void ggf_launch_measure(const LaunchCtx &lc, uint32_t mask, double *out, int kmax) {
  const size_t lds = kmax > 1 ? 4 * (kPairLd * kPairLd + 64) * sizeof(double2) : 0;
  if (mask == 8u) {
    const dim3 grid(lc.n_chains), block(128);
    if (lc.precision == 64) {
      if (kmax > 1) hipLaunchKernelGGL(k_electric<double>, grid, block, lds, lc.stream, lc, out);
      else hipLaunchKernelGGL(k_electric1<double>, grid, block, 0, lc.stream, lc, out);
    } else {
      if (kmax > 1) hipLaunchKernelGGL(k_electric<float>, grid, block, lds, lc.stream, lc, out);
      else hipLaunchKernelGGL(k_electric1<float>, grid, block, 0, lc.stream, lc, out);
    }
    return;
  }
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_measure<double>, dim3(lc.n_chains), dim3(256), lds, lc.stream, lc, mask, out);
  else
    hipLaunchKernelGGL(k_measure<float>, dim3(lc.n_chains), dim3(256), lds, lc.stream, lc, mask, out);
}

// Staging rows of the allocation-free host measurement (ggf_measure_staged): one fixed array per
// GPU, held until the process ends.  Host code never names the array: it takes the address that
// hipGetSymbolAddress returns on each device, once, and passes that to the kernels and copies.
static __device__ __align__(256) double scratch[static_cast<size_t>(GGF_STAGE_MAX_CHAINS_DEV) * GGF_NOBS_DEV];

hipError_t ggf_stage_address(int device, double **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex m;
  static double *addr[kMaxDevices] = {};
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(m);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    double *p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
    if (cur != device) hipSetDevice(cur);
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

