// Device-side data layout and small dense linear algebra for the GGF kernels.
//
// Layout in HBM (one arena per context):
//   * G arena: every chain's inverse G = M(G)^-1, n x n row-major, float64 or
//     float32, chain c at element offset ChainDev::g_off (256-byte aligned).
//   * factor arena: per chain 8 n elements (same type as G): PT[4][n] = -G[U,:]
//     and QT[4][n] = (G[:,U] K)^T of the last accepted flip, consumed by the
//     streaming update kernel.
//   * link arena: int8 link values, chain c at ChainDev::link_off.
//   * per-chain scalars (SoA): log W, S = N/W (complex), sweep counter,
//     accept counters, status flags.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GGF_KMAX_DEV 4
#define GGF_NOBS_DEV 21
#define GGF_MAX_MESON 16
#define GGF_ZN_MAX 64      // largest gauge group Z_N (link values are int8)
#define GGF_ENERGY_STRIDE_DEV (1 + 4 * GGF_KMAX_DEV * GGF_KMAX_DEV)
#define GGF_SENS_STRIDE_DEV 200
#define GGF_BOND_STRIDE_DEV 450   // 2 + 12 + 4 + 3 * 12 * 12

// Per-ansatz constants.  Pair (n, m) of the superposition involves at most
// two patch links (those where B_n or B_m differ from B_0); for each of them
// dg holds the unrotated change gamma^{nm}_link - gamma_b0 of the transition
// covariance of |B_n><B_m| on that link.
struct TensorDev {
  int group, K, pad0, pad1;
  double a[4];          // physical block of the on-site covariance (2x2)
  double b[16];         // physical-virtual block (2x8)
  double d[64];         // virtual block (8x8)
  double x0[4];         // out-in block of the reference bond (2x2)
  double2 w[GGF_KMAX_DEV][GGF_KMAX_DEV];              // lambda_n^* lambda_m <B_m|B_n>
  double2 ov[GGF_KMAX_DEV][GGF_KMAX_DEV];             // <B_m|B_n>
  int nl[GGF_KMAX_DEV][GGF_KMAX_DEV];                 // involved patch links of pair (n,m): 0..2
  int lk[GGF_KMAX_DEV][GGF_KMAX_DEV][2];              // their lattice link indices
  double2 dg[GGF_KMAX_DEV][GGF_KMAX_DEV][2][16];      // 4x4 complex per involved link
  // electric field (Sec. 5.3): mixed occupation of a link's outgoing mode in the
  // transition |ket><bra| of its bond, X = en + (1/2) tr(G_UU O eq O^T), O the link's
  // rotation; reference bond on both sides (en0, eq0), or per involved patch link
  double2 en0;
  double2 eq0[16];
  double2 en[GGF_KMAX_DEV][GGF_KMAX_DEV][2];
  double2 eq[GGF_KMAX_DEV][GGF_KMAX_DEV][2][16];
};

struct ChainDev {
  int L, n, nlinks, tensor;
  int group, K, pad0, pad1;
  size_t g_off;     // element offset of G
  size_t f_off;     // element offset of the factor buffer (8 n elements)
  size_t link_off;  // byte offset of the link values
  size_t scr_off;   // element offset in the float64 refactorisation scratch (set per batch)
  size_t y_off;     // element offset of the pivot-row snapshot of the Gauss-Jordan update (set per batch)
};

// Status flag bits per chain.
#define GGF_FLAG_NONFINITE 1
#define GGF_FLAG_SINGULAR 2

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// mixed with the other counter words and the key, key bumped by Weyl constants.
__host__ __device__ __forceinline__ uint32_t ggf_mulhi(uint32_t a, uint32_t b) {
  return static_cast<uint32_t>((static_cast<uint64_t>(a) * b) >> 32);
}

__host__ __device__ __forceinline__ uint4 ggf_philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = ggf_mulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = ggf_mulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__host__ __device__ __forceinline__ double ggf_u53(uint32_t x0, uint32_t x1) {
  const uint64_t bits = ((static_cast<uint64_t>(x1) << 32) | x0) >> 11;
  return static_cast<double>(bits) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Lattice helpers (site i = x2*L + x1, link l = 2 i + mu, virtual Majorana 8 i + 2 v + t
// with leg v = l 0, u 1, r 2, d 3).
__device__ __forceinline__ int ggf_shift(int i, int L, int d1, int d2) {
  int x1 = i % L, x2 = i / L;
  x1 = (x1 + d1 + L) % L;
  x2 = (x2 + d2 + L) % L;
  return x2 * L + x1;
}

// Majorana indices (out0, out1, in0, in1) of link ell.
__device__ __forceinline__ void ggf_link_u(int ell, int L, int u[4]) {
  const int i = ell >> 1, mu = ell & 1;
  if (mu == 0) {
    const int j = ggf_shift(i, L, 1, 0);
    u[0] = 8 * i + 4; u[1] = 8 * i + 5; u[2] = 8 * j + 0; u[3] = 8 * j + 1;
  } else {
    const int j = ggf_shift(i, L, 0, 1);
    u[0] = 8 * i + 2; u[1] = 8 * i + 3; u[2] = 8 * j + 6; u[3] = 8 * j + 7;
  }
}

// Out-in block of a link with value k: R(2 pi k / N) x0, R = [[c, s], [-s, c]].
__device__ __forceinline__ void ggf_bond_block(const double x0[4], int k, int group, double y[4]) {
  double c = 1.0, s = 0.0;
  if (k != 0) {
    if (group == 2) { c = -1.0; s = 0.0; }
    else { sincospi(2.0 * k / group, &s, &c); }
  }
  y[0] = c * x0[0] + s * x0[2];
  y[1] = c * x0[1] + s * x0[3];
  y[2] = -s * x0[0] + c * x0[2];
  y[3] = -s * x0[1] + c * x0[3];
}

// ---------------------------------------------------------------------------
// Complex helpers (double2 = re, im).
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double den = cabs2(b);
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// Real 4x4: determinant and solve by Gaussian elimination with partial pivoting.
// Solves A X = B in place (A destroyed, B overwritten by X); returns det(A).
__device__ inline double ggf_solve4(double A[16], double B[16]) {
  double det = 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int p = k;
    double best = fabs(A[k * 4 + k]);
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const double v = fabs(A[i * 4 + k]);
      if (v > best) { best = v; p = i; }
    }
    if (p != k) {
      det = -det;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double t = A[k * 4 + j]; A[k * 4 + j] = A[p * 4 + j]; A[p * 4 + j] = t;
        t = B[k * 4 + j]; B[k * 4 + j] = B[p * 4 + j]; B[p * 4 + j] = t;
      }
    }
    const double pv = A[k * 4 + k];
    det *= pv;
    if (pv == 0.0) return 0.0;
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const double f = A[i * 4 + k] / pv;
#pragma unroll
      for (int j = k; j < 4; ++j) A[i * 4 + j] -= f * A[k * 4 + j];
#pragma unroll
      for (int j = 0; j < 4; ++j) B[i * 4 + j] -= f * B[k * 4 + j];
    }
  }
#pragma unroll
  for (int k = 3; k >= 0; --k) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = B[k * 4 + j];
#pragma unroll
      for (int i = k + 1; i < 4; ++i) v -= A[k * 4 + i] * B[i * 4 + j];
      B[k * 4 + j] = v / A[k * 4 + k];
    }
  }
  return det;
}

// Complex Pfaffian of an m x m antisymmetric matrix (leading dimension ld),
// destroyed in place.  Skew Gaussian elimination: per pair step, the largest
// entry below the diagonal of column k is swapped into row/column k+1 (a sign
// flip), the Pfaffian picks up A[k][k+1], and a unit-determinant congruence
// clears row/column k: trailing A += tau v^T - v tau^T, tau = A[k][k+2:]/A[k][k+1],
// v = A[k+2:][k+1].
__device__ inline double2 ggf_cpfaffian(double2 *A, int m, int ld) {
  double2 pf = make_double2(1.0, 0.0);
  for (int k = 0; k + 1 < m; k += 2) {
    int kp = k + 1;
    double best = cabs2(A[(k + 1) * ld + k]);
    for (int i = k + 2; i < m; ++i) {
      const double v = cabs2(A[i * ld + k]);
      if (v > best) { best = v; kp = i; }
    }
    if (kp != k + 1) {
      for (int j = 0; j < m; ++j) {
        const double2 t = A[(k + 1) * ld + j]; A[(k + 1) * ld + j] = A[kp * ld + j]; A[kp * ld + j] = t;
      }
      for (int i = 0; i < m; ++i) {
        const double2 t = A[i * ld + k + 1]; A[i * ld + k + 1] = A[i * ld + kp]; A[i * ld + kp] = t;
      }
      pf = cscale(pf, -1.0);
    }
    const double2 piv = A[k * ld + k + 1];
    if (piv.x == 0.0 && piv.y == 0.0) return make_double2(0.0, 0.0);
    pf = cmul(pf, piv);
    for (int i = k + 2; i < m; ++i) {
      const double2 ti = cdiv(A[k * ld + i], piv);
      const double2 vi = A[i * ld + k + 1];
      for (int j = k + 2; j < m; ++j) {
        const double2 tj = cdiv(A[k * ld + j], piv);
        const double2 vj = A[j * ld + k + 1];
        A[i * ld + j] = cadd(A[i * ld + j], csub(cmul(ti, vj), cmul(vi, tj)));
      }
    }
  }
  return pf;
}

// Complex solve X (I + P Q) = ... helper: invert an m x m complex matrix in
// place (Gauss-Jordan with partial pivoting); returns false when singular.
__device__ inline bool ggf_cinvert(double2 *A, int m, int ld, int *piv) {
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = cabs2(A[k * ld + k]);
    for (int i = k + 1; i < m; ++i) {
      const double v = cabs2(A[i * ld + k]);
      if (v > best) { best = v; p = i; }
    }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int j = 0; j < m; ++j) {
        const double2 t = A[k * ld + j]; A[k * ld + j] = A[p * ld + j]; A[p * ld + j] = t;
      }
    const double2 pv = A[k * ld + k];
    A[k * ld + k] = make_double2(1.0, 0.0);
    for (int j = 0; j < m; ++j) A[k * ld + j] = cdiv(A[k * ld + j], pv);
    for (int i = 0; i < m; ++i) {
      if (i == k) continue;
      const double2 f = A[i * ld + k];
      A[i * ld + k] = make_double2(0.0, 0.0);
      for (int j = 0; j < m; ++j) A[i * ld + j] = csub(A[i * ld + j], cmul(f, A[k * ld + j]));
    }
  }
  for (int k = m - 1; k >= 0; --k)
    if (piv[k] != k)
      for (int i = 0; i < m; ++i) {
        const double2 t = A[i * ld + k]; A[i * ld + k] = A[i * ld + piv[k]]; A[i * ld + piv[k]] = t;
      }
  return true;
}

// Rotated 4x4 change on a link with value k: O dg O^T, O = R(theta) (+) 1_2 acting on (out0,out1).
__device__ inline void ggf_rotate_dg(const double2 dg[16], int k, int group, double2 out[16]) {
  double c = 1.0, s = 0.0;
  if (k != 0) {
    if (group == 2) { c = -1.0; s = 0.0; }
    else { sincospi(2.0 * k / group, &s, &c); }
  }
  const double o[16] = {c, s, 0, 0, -s, c, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  double2 t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double2 v = make_double2(0, 0);
      for (int q = 0; q < 4; ++q) v = cadd(v, cscale(dg[q * 4 + j], o[i * 4 + q]));
      t[i * 4 + j] = v;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double2 v = make_double2(0, 0);
      for (int q = 0; q < 4; ++q) v = cadd(v, cscale(t[i * 4 + q], o[j * 4 + q]));
      out[i * 4 + j] = v;
    }
}
