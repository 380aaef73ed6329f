// Device helpers for the K > 1 cross terms shared by the link-step, measurement
// and block-move kernels: the per-pair patch matrix [[G'_SS, 1], [-1, Delta_SS]]
// whose Pfaffian gives r_nm = Pf(M_nm)/Pf(M_00) (Sec. 5 cross terms, evaluated
// on the Majoranas of the patch links where B_n or B_m differ from B_0).
#pragma once
#include "ggf_device.h"

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

namespace {

constexpr int kPairLd = 16;   // leading dimension of the per-pair 2s x 2s workspace (s <= 8)

// Read access to the current inverse on the Majoranas a pair Pfaffian needs.
// Entries whose both indices are among the nc Majoranas cidx[] are served from
// `cache` (nc x nc, leading dimension 16; the link-step kernel stores there the
// inverse corrected for the flips pending in its window); other entries are
// read from G.
template <typename T>
struct GView {
  const T *G;
  int n;
  const double *cache = nullptr;
  const int *cidx = nullptr;
  int nc = 0;
  __device__ double at(int a, int b) const {
    if (nc > 0) {
      int pa = -1, pb = -1;
      for (int i = 0; i < nc; ++i) {
        if (cidx[i] == a) pa = i;
        if (cidx[i] == b) pb = i;
      }
      if (pa >= 0 && pb >= 0) return cache[pa * 16 + pb];
    }
    return static_cast<double>(G[static_cast<size_t>(a) * n + b]);
  }
};

template <typename T>
__device__ inline GView<T> plain_view(const T *G, int n) {
  return GView<T>{G, n};
}

struct PatchSet {
  int s;
  int idx[8];
};

__device__ inline void pair_set(const TensorDev &Tn, int a, int b, int L, PatchSet &ps) {
  const int nl = Tn.nl[a][b];
  ps.s = 4 * nl;
  for (int l = 0; l < nl; ++l) {
    int u[4];
    ggf_link_u(Tn.lk[a][b][l], L, u);
    for (int q = 0; q < 4; ++q) ps.idx[4 * l + q] = u[q];
  }
}

// Fill W (2s x 2s, leading dimension 16) with [[G'_SS, 1], [-1, Delta_SS]] for pair (a, b).
// G'_SS is G restricted to the pair's patch Majoranas, plus the Woodbury term
// G_SU K G_SU^T of a proposed flip when Kw != nullptr; Delta_SS is the rotated
// change of the transition covariance on each involved link (link ell_prop
// taken at its proposed value k_prop).
template <typename T>
__device__ inline void build_pair_matrix(const TensorDev &Tn, int a, int b, int L, int group, const GView<T> &G,
                                         const int8_t *lk, const int *U, const double *Kw, int ell_prop,
                                         int k_prop, double2 *W, PatchSet &ps) {
  pair_set(Tn, a, b, L, ps);
  const int s = ps.s, m = 2 * s;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double2 v = make_double2(0.0, 0.0);
      if (i < s && j < s) v.x = G.at(ps.idx[i], ps.idx[j]);
      else if (i < s && j == i + s) v.x = 1.0;
      else if (i >= s && j == i - s) v.x = -1.0;
      W[i * kPairLd + j] = v;
    }
  if (Kw != nullptr) {
    double p[8][4];
    for (int i = 0; i < s; ++i)
      for (int q = 0; q < 4; ++q) p[i][q] = G.at(ps.idx[i], U[q]);
    for (int i = 0; i < s; ++i) {
      double t[4];
      for (int q2 = 0; q2 < 4; ++q2) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v += p[i][q] * Kw[q * 4 + q2];
        t[q2] = v;
      }
      for (int j = 0; j < s; ++j) {
        double v = 0.0;
        for (int q2 = 0; q2 < 4; ++q2) v += t[q2] * p[j][q2];
        W[i * kPairLd + j].x += v;
      }
    }
  }
  const int nl = Tn.nl[a][b];
  for (int l = 0; l < nl; ++l) {
    const int link = Tn.lk[a][b][l];
    const int kv = (link == ell_prop) ? k_prop : lk[link];
    double2 blk[16];
    ggf_rotate_dg(Tn.dg[a][b][l], kv, group, blk);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) W[(s + 4 * l + i) * kPairLd + s + 4 * l + j] = blk[i * 4 + j];
  }
}

// r_ab = Pf(M_ab)/Pf(M_00) = (-1)^(s/2) Pf(W); W is destroyed.
__device__ inline double2 pair_ratio(double2 *W, int s) {
  double2 pf = ggf_cpfaffian(W, 2 * s, kPairLd);
  if ((s / 2) & 1) pf = cscale(pf, -1.0);
  return pf;
}

// Lane-parallel forms for one wave (64 lanes) evaluating up to 8 pairs at once,
// 8 lanes per pair; lane gl of a group owns rows gl, gl + 8 of the pair matrix.
// They perform per element the same operations as build_pair_matrix and
// ggf_cpfaffian (bit-identical results, the same pivots).
constexpr int kPairLanes = 8;

// Row ii of ggf_rotate_dg's O dg O^T, by the same operations in the same order.
__device__ inline void rotate_dg_row(const double2 dg[16], int k, int group, int ii, double2 out[4]) {
  double c = 1.0, s = 0.0;
  if (k != 0) {
    if (group == 2) { c = -1.0; s = 0.0; }
    else { sincospi(2.0 * k / group, &s, &c); }
  }
  const double o[16] = {c, s, 0, 0, -s, c, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  double2 t[4];
  for (int j = 0; j < 4; ++j) {
    double2 v = make_double2(0, 0);
    for (int q = 0; q < 4; ++q) v = cadd(v, cscale(dg[q * 4 + j], o[ii * 4 + q]));
    t[j] = v;
  }
  for (int j = 0; j < 4; ++j) {
    double2 v = make_double2(0, 0);
    for (int q = 0; q < 4; ++q) v = cadd(v, cscale(t[q], o[j * 4 + q]));
    out[j] = v;
  }
}

// Rows of the pair matrix of (a, b) with G' = G_II + G_IU K G_UI read from the
// current inverse on the index set I (gI: nI x nI, row stride 16, U first in I).
__device__ inline void build_pair_rows(const TensorDev &Tn, int a, int b, int group, const double *gI,
                                       const int *I, int nI, const int8_t *lk, const double *Kw, int ell_prop,
                                       int k_prop, const PatchSet &ps, double2 *W, int gl) {
  const int s = ps.s, m = 2 * s;
  int pos[8];
  for (int i = 0; i < s; ++i) {
    pos[i] = 0;
    for (int q = 0; q < nI; ++q)
      if (I[q] == ps.idx[i]) pos[i] = q;
  }
  for (int i = gl; i < m; i += kPairLanes) {
    if (i < s) {
      double t[4];
      for (int q2 = 0; q2 < 4; ++q2) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v += gI[pos[i] * 16 + q] * Kw[q * 4 + q2];
        t[q2] = v;
      }
      for (int j = 0; j < s; ++j) {
        double v = 0.0;
        for (int q2 = 0; q2 < 4; ++q2) v += t[q2] * gI[pos[j] * 16 + q2];
        W[i * kPairLd + j] = make_double2(gI[pos[i] * 16 + pos[j]] + v, 0.0);
      }
      for (int j = s; j < m; ++j) W[i * kPairLd + j] = make_double2(j == i + s ? 1.0 : 0.0, 0.0);
    } else {
      for (int j = 0; j < s; ++j) W[i * kPairLd + j] = make_double2(j == i - s ? -1.0 : 0.0, 0.0);
      const int l = (i - s) >> 2, ii = (i - s) & 3;
      const int link = Tn.lk[a][b][l];
      const int kv = (link == ell_prop) ? k_prop : lk[link];
      double2 brow[4];
      rotate_dg_row(Tn.dg[a][b][l], kv, group, ii, brow);
      for (int j = s; j < m; ++j)
        W[i * kPairLd + j] = ((j - s) >> 2) == l ? brow[(j - s) & 3] : make_double2(0.0, 0.0);
    }
  }
}

// Pfaffian of the m x m (m <= 16) skew matrix A (leading dimension kPairLd) by the
// group's 8 lanes; tv: 32 complex of group scratch.  Every lane of the wave must
// call it (it synchronises the workgroup, one wave); lanes of an idle group pass m = 0.
__device__ inline double2 pfaffian_lanes(double2 *A, int m, double2 *tv, int gl) {
  constexpr int ld = kPairLd;
  double2 pf = make_double2(1.0, 0.0);
  bool zero = false;
  for (int k = 0; k < 16; k += 2) {
    const bool live = !zero && k + 1 < m;
    double best = -1.0;
    int kp = k + 1;
    if (live)
      for (int i = k + 1 + gl; i < m; i += kPairLanes) {
        const double v = cabs2(A[i * ld + k]);
        if (v > best) { best = v; kp = i; }
      }
    for (int off = kPairLanes / 2; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, kPairLanes);
      const int oi = __shfl_xor(kp, off, kPairLanes);
      if (ob > best || (ob == best && oi < kp)) { best = ob; kp = oi; }
    }
    const bool sw = live && kp != k + 1;
    __syncthreads();
    if (sw)
      for (int j = gl; j < m; j += kPairLanes) {
        const double2 t = A[(k + 1) * ld + j]; A[(k + 1) * ld + j] = A[kp * ld + j]; A[kp * ld + j] = t;
      }
    __syncthreads();
    if (sw)
      for (int i = gl; i < m; i += kPairLanes) {
        const double2 t = A[i * ld + k + 1]; A[i * ld + k + 1] = A[i * ld + kp]; A[i * ld + kp] = t;
      }
    __syncthreads();
    double2 piv = make_double2(1.0, 0.0);
    if (live) {
      if (sw) pf = cscale(pf, -1.0);
      piv = A[k * ld + k + 1];
      if (piv.x == 0.0 && piv.y == 0.0) zero = true;
      else pf = cmul(pf, piv);
    }
    if (live && !zero)
      for (int x = k + 2 + gl; x < m; x += kPairLanes) {
        tv[x] = cdiv(A[k * ld + x], piv);
        tv[16 + x] = A[x * ld + k + 1];
      }
    __syncthreads();
    if (live && !zero)
      for (int i = k + 2 + gl; i < m; i += kPairLanes) {
        const double2 ti = tv[i], vi = tv[16 + i];
        for (int j = k + 2; j < m; ++j)
          A[i * ld + j] = cadd(A[i * ld + j], csub(cmul(ti, tv[16 + j]), cmul(vi, tv[j])));
      }
    __syncthreads();
  }
  return zero ? make_double2(0.0, 0.0) : pf;
}

__device__ inline void pair_of(int p, int K, int &a, int &b) {
  // enumerate a <= b, skipping (0, 0): p = 0 .. K(K+1)/2 - 2
  int q = p + 1;
  a = 0;
  while (q >= K - a) { q -= K - a; ++a; }
  b = a + q;
}


}  // namespace
