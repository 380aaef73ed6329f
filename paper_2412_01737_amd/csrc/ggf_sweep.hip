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
// Delayed updates (lc.dld > 0): the flips of a window of F link steps are not
// applied at once.  Step t of the window reads the current inverse as
// G - X Y^T (X, Y: 4F columns of length n stored one after another, slots
// 0..t-1 filled); on accept the workgroup writes
// slot t: X[:, 4t..4t+3] = G_cur[:,U] K and Y[:, 4t..4t+3] = G_cur[U,:]^T, so that
// G_cur' = G_cur - G_cur[:,U] K G_cur[U,:]; a rejected or absent step writes
// zeros.  At the end of the window one matrix-core GEMM applies G -= X Y^T
// (rank 4F): one pass over G per window instead of one per accepted flip.
#include "ggf_device.h"
#include "ggf_launch.h"
#include "ggf_pair.h"

namespace {

constexpr int kDelaySlotsMax = 32;   // window length F <= 32 (rank 4F <= 128)

template <typename T>
__global__ __launch_bounds__(256) void k_ratio(LaunchCtx lc, int ell, int parity, int t) {
  extern __shared__ double2 s_work[];
  __shared__ double s_K[16];
  __shared__ double s_GI[16 * 16];     // current inverse on the link's and the patch links' Majoranas
  __shared__ int s_I[16];
  __shared__ int s_nI;
  __shared__ double s_xu[4][4 * kDelaySlotsMax], s_yu[4][4 * kDelaySlotsMax];   // X[U,:r], Y[U,:r]
  __shared__ double s_rho, s_u;
  __shared__ int s_kn, s_acc;
  __shared__ double2 s_r[16];
  const int c = blockIdx.x;
  if (c == 0 && threadIdx.x == 0) lc.acc_cnt[parity ^ 1] = 0;
  const ChainDev ch = lc.chains[c];
  const int n = ch.n;
  const bool delayed = lc.dld > 0;
  const int r = delayed ? 4 * t : 0;
  T *X = delayed ? static_cast<T *>(lc.X) + lc.x_off[c] : nullptr;
  T *Y = delayed ? static_cast<T *>(lc.Y) + lc.x_off[c] : nullptr;
  // a step without an accepted flip leaves zeros in its slot of the window
  auto zero_slot = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        X[static_cast<size_t>(r + q) * n + j] = static_cast<T>(0);
        Y[static_cast<size_t>(r + q) * n + j] = static_cast<T>(0);
      }
  };
  if (ell >= ch.nlinks) {
    if (delayed) {
      if (t == 0 && threadIdx.x == 0) lc.pend[c] = 0;
      zero_slot();
    }
    return;
  }
  const TensorDev &Tn = lc.tensors[ch.tensor];
  const T *G = static_cast<const T *>(lc.G) + ch.g_off;
  int8_t *lk = lc.links + ch.link_off;
  int U[4];
  ggf_link_u(ell, ch.L, U);
  for (int i = threadIdx.x; i < 4 * r; i += blockDim.x) {
    const int q = i / r, s = i - q * r;
    s_xu[q][s] = static_cast<double>(X[static_cast<size_t>(s) * n + U[q]]);
    s_yu[q][s] = static_cast<double>(Y[static_cast<size_t>(s) * n + U[q]]);
  }
  const int K = ch.K;
  const int npairs = K * (K + 1) / 2 - 1;
  if (threadIdx.x == 0) {
    // index set: U first, then the Majoranas of every patch link of the superposition
    int m = 0;
    for (int q = 0; q < 4; ++q) s_I[m++] = U[q];
    for (int p = 0; p < npairs; ++p) {
      int a, b;
      pair_of(p, K, a, b);
      for (int l = 0; l < Tn.nl[a][b]; ++l) {
        int u4[4];
        ggf_link_u(Tn.lk[a][b][l], ch.L, u4);
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
  for (int e = threadIdx.x; e < nI * nI; e += blockDim.x) {
    const int i = e / nI, j = e - i * nI;
    const int a = s_I[i], b = s_I[j];
    double v = static_cast<double>(G[static_cast<size_t>(a) * n + b]);
    for (int s = 0; s < r; ++s)
      v -= static_cast<double>(X[static_cast<size_t>(s) * n + a]) * static_cast<double>(Y[static_cast<size_t>(s) * n + b]);
    s_GI[i * 16 + j] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int kold = lk[ell];
    const uint4 x = ggf_philox(make_uint4(static_cast<uint32_t>(c), lc.sweep[c], static_cast<uint32_t>(ell), 0u),
                               lc.key0, lc.key1);
    const int kn = (ch.group == 2) ? (1 - kold) : (kold + 1 + static_cast<int>(x.z & 1u)) % 3;
    double yo[4], yn[4];
    ggf_bond_block(Tn.x0, kold, ch.group, yo);
    ggf_bond_block(Tn.x0, kn, ch.group, yn);
    const double X0 = yn[0] - yo[0], X1 = yn[1] - yo[1], X2 = yn[2] - yo[2], X3 = yn[3] - yo[3];
    const double dM[16] = {0, 0, X0, X1, 0, 0, X2, X3, -X0, -X2, 0, 0, -X1, -X3, 0, 0};
    double A[16], Ai[16];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double v = (a == b) ? 1.0 : 0.0;
        for (int q = 0; q < 4; ++q) v += s_GI[a * 16 + q] * dM[q * 4 + b];
        A[a * 4 + b] = v;
        Ai[a * 4 + b] = (a == b) ? 1.0 : 0.0;
      }
    const double rho = ggf_solve4(A, Ai);      // Ai <- (1 + G_UU dM)^-1
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v += dM[a * 4 + q] * Ai[q * 4 + b];
        s_K[a * 4 + b] = v;
      }
    s_rho = rho;
    s_kn = kn;
    s_u = ggf_u53(x.x, x.y);
  }
  __syncthreads();
  if (K > 1) {
    if (threadIdx.x < npairs) {
      int a, b;
      pair_of(threadIdx.x, K, a, b);
      PatchSet ps;
      double2 *W = s_work + threadIdx.x * kPairLd * kPairLd;
      GView<T> gv{G, n, X, Y, r};
      gv.cache = s_GI;
      gv.cidx = s_I;
      gv.nc = nI;
      build_pair_matrix(Tn, a, b, ch.L, ch.group, gv, lk, U, s_K, ell, s_kn, W, ps);
      s_r[threadIdx.x] = pair_ratio(W, ps.s);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double rho = s_rho;
    double2 snew = make_double2(1.0, 0.0);
    double sratio = 1.0;
    if (K > 1) {
      double sv = Tn.w[0][0].x;
      for (int p = 0; p < npairs; ++p) {
        int a, b;
        pair_of(p, K, a, b);
        const double2 tt = cmul(Tn.w[a][b], s_r[p]);
        sv += (a == b) ? tt.x : 2.0 * tt.x;
      }
      snew = make_double2(sv, 0.0);
      sratio = sv / lc.sfac[c].x;
    }
    const bool bad = !isfinite(rho) || !isfinite(sratio) || rho < -1e-6;
    const double R = (rho > 0.0 ? sqrt(rho) : 0.0) * sratio;
    const bool accept = !bad && (s_u < R);
    lc.prop_total[c] += 1;
    if (bad) lc.flags[c] |= GGF_FLAG_NONFINITE;
    if (accept) {
      lk[ell] = static_cast<int8_t>(s_kn);
      lc.logw[c] += 0.5 * log(rho);
      lc.sfac[c] = snew;
      lc.acc_since[c] += 1;
      lc.acc_total[c] += 1;
      if (delayed) {
        lc.pend[c] = t + 1;
      } else {
        const int slot = atomicAdd(lc.acc_cnt + parity, 1);
        lc.acc_list[slot] = c;
      }
    } else if (delayed && t == 0) {
      lc.pend[c] = 0;
    }
    s_acc = accept ? 1 : 0;
  }
  __syncthreads();
  const int u0 = U[0], u1 = U[1], u2 = U[2], u3 = U[3];
  if (delayed) {
    if (!s_acc) {
      zero_slot();
      return;
    }
    // slot t: X = G_cur[:,U] K, Y = G_cur[U,:]^T, with G_cur = G - X Y^T over slots 0..t-1
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const T *gj = G + static_cast<size_t>(j) * n;
      double gc[4] = {static_cast<double>(gj[u0]), static_cast<double>(gj[u1]), static_cast<double>(gj[u2]),
                      static_cast<double>(gj[u3])};
      double gr[4] = {static_cast<double>(G[static_cast<size_t>(u0) * n + j]),
                      static_cast<double>(G[static_cast<size_t>(u1) * n + j]),
                      static_cast<double>(G[static_cast<size_t>(u2) * n + j]),
                      static_cast<double>(G[static_cast<size_t>(u3) * n + j])};
      for (int s0 = 0; s0 < r; s0 += 4) {     // r is a multiple of 4: four slots' loads in flight
        double xs[4], ys[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          xs[d] = static_cast<double>(X[static_cast<size_t>(s0 + d) * n + j]);
          ys[d] = static_cast<double>(Y[static_cast<size_t>(s0 + d) * n + j]);
        }
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            gc[q] -= xs[d] * s_yu[q][s0 + d];
            gr[q] -= s_xu[q][s0 + d] * ys[d];
          }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        X[static_cast<size_t>(r + b) * n + j] = static_cast<T>(
            gc[0] * s_K[0 * 4 + b] + gc[1] * s_K[1 * 4 + b] + gc[2] * s_K[2 * 4 + b] + gc[3] * s_K[3 * 4 + b]);
        Y[static_cast<size_t>(r + b) * n + j] = static_cast<T>(gr[b]);
      }
    }
    return;
  }
  if (!s_acc) return;
  // Woodbury with the stored rows and columns: G' = G - G[:,U] K G[U,:].
  // (Substituting -G[U,:]^T for G[:,U] would assume exact antisymmetry; rounding
  // breaks it and the symmetric part of the error then grows with every flip.)
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
  if (c < lc.n_chains) lc.sweep[c] += 1u;
  if (c < 2) lc.acc_cnt[c] = 0;   // every sweep starts with both accepted counters cleared
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

// Observables of one chain per workgroup (Sec. 2.3, 5.1, 5.2).  Fermionic
// two-point functions: Gamma_out = A + B M^-1 B^T (per pair (a, b) of the
// superposition with M_ab^-1 = G - G_S Y_ab G_S^T, Y_ab = Delta (1 + G_SS Delta)^-1),
// <c_p c_q> = -i Gamma_out, weights lambda_a^* lambda_b <B_b|B_a> r_ab / S.
template <typename T>
__global__ __launch_bounds__(256) void k_measure(LaunchCtx lc, uint32_t mask, double *out) {
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
    }
  }
  __syncthreads();
  double Sv = 0.0;
  for (int p = 0; p < npairs; ++p) Sv += s_om[p].x;
  const double invS = 1.0 / Sv;
  double acc[GGF_NOBS_DEV];
  for (int q = 0; q < GGF_NOBS_DEV; ++q) acc[q] = 0.0;
  const int nmes = min(L / 2, GGF_MAX_MESON);
  for (int x = threadIdx.x; x < V; x += blockDim.x) {
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
        double base[4] = {0, 0, 0, 0};   // (b G_xy b^T)[p][q]
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
        if (r == 0) {
          base[0] += Tn.a[0]; base[1] += Tn.a[1]; base[2] += Tn.a[2]; base[3] += Tn.a[3];
        }
        double2 tot = make_double2(0.0, 0.0);
        for (int pr = 0; pr < npairs; ++pr) {
          double2 gm[4] = {make_double2(base[0], 0), make_double2(base[1], 0), make_double2(base[2], 0),
                           make_double2(base[3], 0)};
          const int s = s_s[pr];
          if (s > 0) {
            double vx[2][8], vy[2][8];
            for (int q = 0; q < s; ++q) {
              const int col = s_S[pr][q];
              double ax0 = 0, ax1 = 0, ay0 = 0, ay1 = 0;
              for (int i = 0; i < 8; ++i) {
                const double gx = static_cast<double>(G[static_cast<size_t>(8 * x + i) * n + col]);
                const double gy = static_cast<double>(G[static_cast<size_t>(8 * y + i) * n + col]);
                ax0 += Tn.b[i] * gx; ax1 += Tn.b[8 + i] * gx;
                ay0 += Tn.b[i] * gy; ay1 += Tn.b[8 + i] * gy;
              }
              vx[0][q] = ax0; vx[1][q] = ax1; vy[0][q] = ay0; vy[1][q] = ay1;
            }
            // + v_x Y v_y^T   (G_Sy = -G_yS^T makes -G_xS Y G_Sy = + v_x Y v_y^T)
            for (int pp = 0; pp < 2; ++pp)
              for (int qq = 0; qq < 2; ++qq) {
                double2 v = make_double2(0, 0);
                for (int i = 0; i < s; ++i)
                  for (int j = 0; j < s; ++j) v = cadd(v, cscale(s_Y[pr][i * 8 + j], vx[pp][i] * vy[qq][j]));
                gm[pp * 2 + qq] = cadd(gm[pp * 2 + qq], v);
              }
          }
          double2 f;
          if (r == 0) {
            f = cscale(cadd(make_double2(1.0, 0.0), gm[1]), 0.5);    // (1 + Gamma_out[x0,x1]) / 2
          } else {
            // <phi_x^+ phi_y> = 1/4 [<c0c0> + i<c0c1> - i<c1c0> + <c1c1>], <c_p c_q> = -i Gamma
            const double2 m00 = make_double2(gm[0].y, -gm[0].x), m01 = make_double2(gm[1].y, -gm[1].x);
            const double2 m10 = make_double2(gm[2].y, -gm[2].x), m11 = make_double2(gm[3].y, -gm[3].x);
            double2 bil = cadd(m00, m11);
            bil = cadd(bil, make_double2(-m01.y, m01.x));
            bil = csub(bil, make_double2(-m10.y, m10.x));
            f = cscale(bil, 0.5);                                       // 2 * (1/4) * bilinear
          }
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
  for (int q = 0; q < GGF_NOBS_DEV; ++q) {
    const double t = block_sum(acc[q], red);
    if (threadIdx.x == 0) out[static_cast<size_t>(c) * GGF_NOBS_DEV + q] = t / V;
  }
  if (threadIdx.x == 0) out[static_cast<size_t>(c) * GGF_NOBS_DEV + 3] =
      (mask & 2u) ? lc.logw[c] + (K > 1 ? log(Sv) : 0.0) : 0.0;
}

}  // namespace

static size_t pair_lds(int kmax) {
  const int np = kmax * (kmax + 1) / 2 - 1;
  return np > 0 ? static_cast<size_t>(np) * kPairLd * kPairLd * sizeof(double2) : 0;
}

void ggf_launch_ratio(const LaunchCtx &lc, int ell, int parity, int kmax, int t, int n_max) {
  const size_t lds = pair_lds(kmax);
  // (one wave per chain was measured slower on 8x8 float64: the pending-factor reads of an
  // accepted flip need the full workgroup)
  const int threads = 256;
  (void)n_max;
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_ratio<double>, dim3(lc.n_chains), dim3(threads), lds, lc.stream, lc, ell, parity, t);
  else
    hipLaunchKernelGGL(k_ratio<float>, dim3(lc.n_chains), dim3(threads), lds, lc.stream, lc, ell, parity, t);
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

void ggf_launch_measure(const LaunchCtx &lc, uint32_t mask, double *out, int kmax) {
  const size_t lds = kmax > 1 ? 4 * (kPairLd * kPairLd + 64) * sizeof(double2) : 0;
  if (lc.precision == 64)
    hipLaunchKernelGGL(k_measure<double>, dim3(lc.n_chains), dim3(256), lds, lc.stream, lc, mask, out);
  else
    hipLaunchKernelGGL(k_measure<float>, dim3(lc.n_chains), dim3(256), lds, lc.stream, lc, mask, out);
}
