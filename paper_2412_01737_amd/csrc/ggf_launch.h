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
  unsigned long long *ties;      // decisions with |u - R| < 1e-9 R (rounding of R could change them)
  int *cursor;                   // balanced sweeps: each chain's next link (nullptr: lock-step link steps)
  double *max_drift;
  double *ldet;
  int *flags;
  int *acc_list;                 // compacted accepted chains of the current link step
  int *acc_cnt;                  // [2] double-buffered accepted counts
  double *scratch;               // float64 refactorisation scratch
  // delayed updates (dly = window length F > 0): the flips accepted so far in
  // the window are the Majoranas A (dU, 4 per flip, dr[c] of them) with their
  // link changes dX (2x2 per flip); the current inverse is
  // G - G[:,A] W G[A,:], W = dM_A Binv, Binv = (1 + G_AA dM_A)^-1 (float64,
  // dBinv with leading dimension GGF_BLOCK_RMAX; W is never formed);
  // chains with a flip pending are listed in acc_list, dcnt[window parity] of them
  int dly;
  int nidx;                      // largest index set of a link step (4 .. 16 Majoranas)
  int *dU, *dr, *dcnt;
  double *dBinv, *dX;
  // rows of the stored G of the pending Majoranas, P = G[A,:] (128 x n per chain, type
  // of G, at dP_off[c]): copied by the link steps (K = 1) or the flush, read by the flush
  void *dP;
  const size_t *dP_off;
  uint32_t key0, key1;
  int n_chains;
  // which chains the window-flush kernels meet: bit 0 some chain's n is a multiple of
  // GGF_WINDOW_TILE (every tile full), bit 1 some chain's n is not
  int tile_kinds;
};

#define GGF_WINDOW_TILE 64

void ggf_launch_assemble(const LaunchCtx &lc, const int *list, int count, int max_sites);
void ggf_launch_gj(const LaunchCtx &lc, const int *list, int count, int n_max, int nb, int *piv,
                   int *perm, size_t piv_stride, double *ybuf);
void ggf_launch_store(const LaunchCtx &lc, const int *list, int count, int n_max, const int *perm,
                      size_t piv_stride);
void ggf_launch_post(const LaunchCtx &lc, const int *list, int count, int is_refresh);

// One link step: ratio + decision + factors, then the streaming rank-4 update
// (or, with delayed updates, the factors of window slot t).
void ggf_launch_ratio(const LaunchCtx &lc, int ell, int parity, int kmax, int t, int wp);
// Delayed updates, end of a window of parity wp: G -= G[:,A] W G[A,:] for every
// listed chain, evaluated on the upper triangle and mirrored (P = G[A,:] in lc.dP,
// copied by the link steps, or by the flush itself when snapshot is set).
void ggf_launch_window_flush(const LaunchCtx &lc, int wp, int grid, bool snapshot);
void ggf_launch_update(const LaunchCtx &lc, int parity, int grid, int tiles, int nt);
void ggf_launch_end_sweep(const LaunchCtx &lc);
void ggf_launch_hot_start(const LaunchCtx &lc, int max_links);
void ggf_launch_sfac(const LaunchCtx &lc, const int *list, int count, int kmax);
void ggf_launch_measure(const LaunchCtx &lc, uint32_t mask, double *out, int kmax);
// Couplings of the gauged Hamiltonian (hopping, chemical, staggered mass, plaquette, electric).
struct EnergyCp {
  double t, mu, m, kb, ke;
};
void ggf_launch_energy(const LaunchCtx &lc, const EnergyCp &cp, double *out, int kmax);
void ggf_launch_bond_rows(const LaunchCtx &lc, const EnergyCp &cp, double *out);
// Sensitivities of Re E_loc and log N to the on-site covariance (K = 1 chains, L <= 32);
// max_group: the largest link group among the chains.
void ggf_launch_sens(const LaunchCtx &lc, const EnergyCp &cp, double *out, int max_sites, int max_group);
// K > 1: per pair, each chain's weighted contribution accumulated into out, using the chains' energy
// rows erows; M_ab^-1 is formed explicitly in scratch when nmax <= 512, else applied as G plus the
// rank <= 8 correction whose factors are kept in scratch.
// Scratch bytes of ggf_launch_sens_pairs: the pair inverses M_ab^-1 (complex nmax x nmax per chain) when
// nmax <= 512, else the correction tables (A, AY, Ab: 26 nmax doubles per chain).
size_t ggf_sens_pairs_scratch(int n_chains, int nmax);
void ggf_launch_sens_pairs(const LaunchCtx &lc, const EnergyCp &cp, void *scratch, int nmax, const double *erows,
                           double *out, int kmax);
int ggf_launch_probe(int mode, void *a, void *b, size_t bytes, int grid, hipStream_t s);
// Staging array of the allocation-free host measurement: GGF_STAGE_MAX_CHAINS x GGF_NOBS_DEV doubles per
// GPU, a fixed device array; its address on `device` (looked up once per device).
#define GGF_STAGE_MAX_CHAINS_DEV 16384
hipError_t ggf_stage_address(int device, double **ptr);
