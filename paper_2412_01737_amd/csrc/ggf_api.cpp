// C ABI of the GGF Monte Carlo library: context, ansatz registration, chain
// storage, sweep orchestration and read-back.  Device work is in
// ggf_factor.hip (refactorisation) and ggf_sweep.hip (link steps, observables).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ggf.h"
#include "ggf_device.h"
#include "ggf_launch.h"
#include "ggf_nn.h"

static_assert(GGF_NOBS == GGF_NOBS_DEV, "observable slot counts of the ABI and the kernels differ");
static_assert(GGF_KMAX == GGF_KMAX_DEV, "superposition sizes of the ABI and the kernels differ");
static_assert(GGF_ENERGY_STRIDE == GGF_ENERGY_STRIDE_DEV, "energy row lengths of the ABI and the kernels differ");
static_assert(GGF_SENS_STRIDE == GGF_SENS_STRIDE_DEV, "sensitivity row lengths of the ABI and the kernels differ");
static_assert(GGF_STAGE_MAX_CHAINS == GGF_STAGE_MAX_CHAINS_DEV, "staging capacities of the ABI and the kernels differ");

typedef std::complex<double> cplx;

namespace {

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct HostBonds;   // an ansatz's bonds, patch links and amplitudes on the host (defined below)

struct ggf_ctx {
  int device = 0;
  std::string err;
  double *stage = nullptr;       // this device's staging array of ggf_measure_staged (fixed, never freed)
  hipError_t stage_err = hipSuccess;
  std::vector<TensorDev> tensors;
  std::vector<HostBonds> bonds;  // host data of each tensor, for ggf_set_bond
  TensorDev *tensors_dev = nullptr;
  size_t tensors_cap = 0;

  // chains
  int n_chains = 0, precision = 64, refresh_every = 0, kmax = 1, max_links = 0, n_max = 0;
  int nidx = 4;   // largest index set of a link step (Majoranas)
  int tile_kinds = 0;            // bit 0: some n % GGF_WINDOW_TILE == 0, bit 1: some other n
  uint64_t seed = 0;
  std::vector<ChainDev> chains;
  std::vector<unsigned long long> recoveries;
  ChainDev *chains_dev = nullptr;
  void *G = nullptr, *F = nullptr;
  int8_t *links = nullptr;
  double *logw = nullptr, *max_drift = nullptr, *ldet = nullptr;
  double2 *sfac = nullptr;
  uint32_t *sweep = nullptr, *acc_since = nullptr;
  unsigned long long *acc_total = nullptr, *prop_total = nullptr, *refreshes = nullptr, *ties = nullptr;
  int *cursor = nullptr;         // each chain's next link within its sweep (balanced sweeps)
  int *flags = nullptr, *acc_list = nullptr, *acc_cnt = nullptr;
  double *scratch = nullptr;
  size_t scratch_elems = 0;
  double *ybuf = nullptr;        // pivot-row snapshots of the Gauss-Jordan update
  size_t ybuf_elems = 0;
  int *piv = nullptr, *perm = nullptr, *list_dev = nullptr;
  size_t piv_stride = 0;
  std::vector<void *> allocs;

  // options
  int opt_update_grid = 0, opt_update_tiles = 0, opt_graph = 0, opt_gj_nb = 0, opt_time_update = 0, opt_update_nt = 1;
  int opt_delay = -1;            // window of delayed updates in link steps (0 = immediate, -1 = automatic)
  int opt_flush_grid = 0;        // workgroups of the window flush (0 = library default)
  int opt_balance = 0;           // 1: balanced sweeps (every chain steps its own link cursor at every link step)
  int opt_block_pend = GGF_BLOCK_RMAX;   // delayed block moves: largest pending rank (0 = apply each move at once)
  int opt_block_rho = 65536;     // move rate of the block proposal in units of 1/65536
  long long opt_scratch_mb = 0;

  // graph replay
  hipStream_t own_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;

  // learned block proposal (network state survives re-initialised chains)
  int nn_P = 0, nn_adam_t = 0, nn_nslices = 256, nn_cap = 0;
  uint32_t nn_step = 0;
  float *nn_p = nullptr, *nn_m = nullptr, *nn_v = nullptr, *nn_g = nullptr, *nn_gpart = nullptr, *nn_logits = nullptr;
  uint16_t *nn_wq = nullptr;
  double *nn_lpart = nullptr, *nn_loss = nullptr;
  int *nn_ex_chain = nullptr, *nn_ex_patch = nullptr;
  std::vector<void *> nn_allocs;
  // block-move buffers (tied to the chains)
  double *blk_A = nullptr, *blk_W = nullptr;
  void *blk_D = nullptr;
  size_t *blk_doff = nullptr;
  int *blk_U = nullptr, *blk_r = nullptr;
  unsigned long long *blk_prop = nullptr, *blk_acc = nullptr;
  // delayed block moves: the decision's move and its products with the pending moves
  double *blk_E = nullptr, *blk_F = nullptr, *blk_Wn = nullptr;
  int *blk_Un = nullptr, *blk_rn = nullptr, *blk_mode = nullptr;

  // delayed-update state (tied to the chains; with the block-move buffers): link changes of
  // the pending flips, window list counters
  double *dly_dX = nullptr;
  int *dly_cnt = nullptr;

  // update timing
  std::vector<hipEvent_t> tev, rev;   // update / ratio kernel events
  int timed_launches = 0;        // update event pairs recorded by the last record_sweep
  double last_ratio_ms = 0.0;
  long long last_ratio_launches = 0;
  double last_update_ms = 0.0;
  long long last_launches = 0, last_flips = 0;
};

namespace {

ggf_status fail(ggf_ctx *ctx, ggf_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                               \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, GGF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Two-mode even bond states.  A pure even state a|00> + b|11> (|11> = psi_out^+ psi_in^+|0>)
// is the ground state of H = -(i/4) sum Gamma_ab c_a c_b restricted to the even sector,
// H = [[h, z], [z^*, -h]] with h = (g01 + g23)/2 and z = (g03 + g12)/2 + i (g02 - g13)/2.
// Matrix elements of the bilinears c_a c_b (a < b) in the even basis (|00>, |11>):
//   c0c1 = c2c3 = diag(i, -i); c0c2 = [[0,-1],[1,0]]; c0c3 = c1c2 = [[0,i],[i,0]]; c1c3 = [[0,1],[-1,0]].
struct Even2 {
  cplx a, b;
};

void bilinear(int p, int q, cplx m[2][2]) {
  const cplx I(0, 1);
  m[0][0] = m[0][1] = m[1][0] = m[1][1] = 0.0;
  if ((p == 0 && q == 1) || (p == 2 && q == 3)) { m[0][0] = I; m[1][1] = -I; }
  else if (p == 0 && q == 2) { m[0][1] = -1.0; m[1][0] = 1.0; }
  else if ((p == 0 && q == 3) || (p == 1 && q == 2)) { m[0][1] = I; m[1][0] = I; }
  else if (p == 1 && q == 3) { m[0][1] = 1.0; m[1][0] = -1.0; }
}

// (i/2) <bra|[c_p,c_q]|ket> / <bra|ket> for all p, q (4x4).
void transition_cov(const Even2 &bra, const Even2 &ket, cplx out[16]) {
  const cplx ov = std::conj(bra.a) * ket.a + std::conj(bra.b) * ket.b;
  for (int i = 0; i < 16; ++i) out[i] = 0.0;
  for (int p = 0; p < 4; ++p)
    for (int q = p + 1; q < 4; ++q) {
      cplx m[2][2];
      bilinear(p, q, m);
      const cplx e = std::conj(bra.a) * (m[0][0] * ket.a + m[0][1] * ket.b) +
                     std::conj(bra.b) * (m[1][0] * ket.a + m[1][1] * ket.b);
      const cplx g = cplx(0, 1) * e / ov;   // [c_p, c_q] = 2 c_p c_q for p != q
      out[p * 4 + q] = g;
      out[q * 4 + p] = -g;
    }
}

// Response of a link's bond operator |ket><bra| to a phase exp(i theta n_out) on the
// outgoing mode of the bra side (Sec. 5.3, overlaps of configurations that differ on
// one link).  The overlap and the Gaussian trace are affine in e^(i theta); their
// slope at theta = 0, divided by i and by the overlap, is
//   nbar = <bra|n_out|ket> / <bra|ket>,
//   Q_pq = i <bra|n_out c_p c_q|ket> / <bra|ket> - Gamma_pq nbar   (p != q),
// the derivative of the transition covariance Gamma.  n_out is |11><11| in the even basis.
void occupation_response(const Even2 &bra, const Even2 &ket, cplx &nbar, cplx q_out[16]) {
  const cplx ov = std::conj(bra.a) * ket.a + std::conj(bra.b) * ket.b;
  nbar = std::conj(bra.b) * ket.b / ov;
  cplx g[16];
  transition_cov(bra, ket, g);
  for (int i = 0; i < 16; ++i) q_out[i] = 0.0;
  for (int p = 0; p < 4; ++p)
    for (int q = p + 1; q < 4; ++q) {
      cplx m[2][2];
      bilinear(p, q, m);
      const cplx e = std::conj(bra.b) * (m[1][0] * ket.a + m[1][1] * ket.b);
      const cplx v = cplx(0, 1) * e / ov - g[p * 4 + q] * nbar;
      q_out[p * 4 + q] = v;
      q_out[q * 4 + p] = -v;
    }
}

void store_response(const Even2 &bra, const Even2 &ket, double2 &en, double2 eq[16]) {
  cplx nb, q[16];
  occupation_response(bra, ket, nb, q);
  en = make_double2(nb.real(), nb.imag());
  for (int i = 0; i < 16; ++i) eq[i] = make_double2(q[i].real(), q[i].imag());
}

bool even_state(const double *g, Even2 &st, std::string &why) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      if (std::fabs(g[i * 4 + j] + g[j * 4 + i]) > 1e-10) { why = "bond covariance is not antisymmetric"; return false; }
  const double h = 0.5 * (g[0 * 4 + 1] + g[2 * 4 + 3]);
  const cplx z(0.5 * (g[0 * 4 + 3] + g[1 * 4 + 2]), 0.5 * (g[0 * 4 + 2] - g[1 * 4 + 3]));
  const double e = std::sqrt(h * h + std::norm(z));
  cplx v0 = z, v1 = -(h + e);
  if (std::abs(h + e) < 0.5) { v0 = e - h; v1 = -std::conj(z); }
  const double nrm = std::sqrt(std::norm(v0) + std::norm(v1));
  if (!(nrm > 0)) { why = "bond covariance has no even ground state"; return false; }
  st.a = v0 / nrm;
  st.b = v1 / nrm;
  cplx back[16];
  transition_cov(st, st, back);
  for (int i = 0; i < 16; ++i)
    if (std::abs(back[i] - g[i]) > 1e-8) { why = "bond covariance is not a pure even-parity state"; return false; }
  return true;
}

}  // namespace

// Host copy of an ansatz's bonds (phase-fixed states), patch links and amplitudes, kept per tensor
// so that a bond or lambda can be replaced later.
struct HostBonds {
  std::vector<Even2> bk;      // bk[0] = reference bond
  std::vector<cplx> cc;       // lambda_k
  std::vector<int> patch;     // patch_link[k]
  double g0[16];              // reference bond covariance
};

namespace {

// The pair tables of a tensor from its bonds: per (n, m) the involved patch links, the change of
// their transition covariance from the reference bond, the electric responses, <B_m|B_n> and
// lambda_n^* lambda_m <B_m|B_n>.
bool fill_pairs(TensorDev &t, const HostBonds &hb, std::string &why) {
  const int K = t.K;
  store_response(hb.bk[0], hb.bk[0], t.en0, t.eq0);
  for (int n = 0; n < K; ++n)
    for (int m = 0; m < K; ++m) {
      int links[2], cnt = 0;
      if (n > 0) links[cnt++] = hb.patch[n];
      if (m > 0 && !(cnt == 1 && links[0] == hb.patch[m])) links[cnt++] = hb.patch[m];
      cplx ovl = 1.0;
      t.nl[n][m] = cnt;
      for (int l = 0; l < cnt; ++l) {
        const Even2 &ket = (n > 0 && hb.patch[n] == links[l]) ? hb.bk[n] : hb.bk[0];
        const Even2 &bra = (m > 0 && hb.patch[m] == links[l]) ? hb.bk[m] : hb.bk[0];
        const cplx o = std::conj(bra.a) * ket.a + std::conj(bra.b) * ket.b;
        if (std::abs(o) < 1e-14) { why = "vanishing bond overlap"; return false; }
        ovl *= o;
        cplx g[16];
        transition_cov(bra, ket, g);
        t.lk[n][m][l] = links[l];
        for (int q = 0; q < 16; ++q)
          t.dg[n][m][l][q] = make_double2((g[q] - hb.g0[q]).real(), (g[q] - hb.g0[q]).imag());
        store_response(bra, ket, t.en[n][m][l], t.eq[n][m][l]);
      }
      const cplx w = std::conj(hb.cc[n]) * hb.cc[m] * ovl;
      t.w[n][m] = make_double2(w.real(), w.imag());
      t.ov[n][m] = make_double2(ovl.real(), ovl.imag());
    }
  return true;
}

bool check_local(const double *g, std::string &why) {
  for (int i = 0; i < 10; ++i)
    for (int j = 0; j < 10; ++j)
      if (std::fabs(g[i * 10 + j] + g[j * 10 + i]) > 1e-10) { why = "gamma_loc is not antisymmetric"; return false; }
  for (int i = 0; i < 10; ++i)
    for (int j = 0; j < 10; ++j) {
      double v = 0;
      for (int k = 0; k < 10; ++k) v += g[i * 10 + k] * g[k * 10 + j];
      if (std::fabs(v + (i == j ? 1.0 : 0.0)) > 1e-8) { why = "gamma_loc is not pure (Gamma^2 != -1)"; return false; }
    }
  return true;
}

template <typename T>
T *dalloc(ggf_ctx *ctx, size_t count, hipError_t &e) {
  void *p = nullptr;
  if (e != hipSuccess) return nullptr;   // an earlier allocation of the batch failed: keep its error
  e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) {
    ctx->allocs.push_back(p);
    e = hipMemset(p, 0, std::max<size_t>(count, 1) * sizeof(T));
  }
  return static_cast<T *>(p);
}

void free_chains(ggf_ctx *ctx) {
  if (ctx->graph_exec) { hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
  for (void *p : ctx->allocs) hipFree(p);
  ctx->allocs.clear();
  ctx->blk_A = ctx->blk_W = nullptr;
  ctx->blk_D = nullptr;
  ctx->dly_dX = nullptr;
  ctx->dly_cnt = nullptr;
  ctx->blk_doff = nullptr;
  ctx->blk_U = ctx->blk_r = nullptr;
  ctx->blk_prop = ctx->blk_acc = nullptr;
  ctx->blk_E = ctx->blk_F = ctx->blk_Wn = nullptr;
  ctx->blk_Un = ctx->blk_rn = ctx->blk_mode = nullptr;
  ctx->n_chains = 0;
  ctx->chains.clear();
  ctx->G = ctx->F = nullptr;
  ctx->scratch = nullptr;
  if (ctx->ybuf) hipFree(ctx->ybuf);
  ctx->ybuf = nullptr;
  ctx->ybuf_elems = 0;
}

LaunchCtx launch_ctx(ggf_ctx *ctx, hipStream_t s) {
  LaunchCtx lc;
  lc.stream = s;
  lc.precision = ctx->precision;
  lc.chains = ctx->chains_dev;
  lc.tensors = ctx->tensors_dev;
  lc.G = ctx->G;
  lc.F = ctx->F;
  lc.links = ctx->links;
  lc.logw = ctx->logw;
  lc.sfac = ctx->sfac;
  lc.sweep = ctx->sweep;
  lc.acc_since = ctx->acc_since;
  lc.acc_total = ctx->acc_total;
  lc.prop_total = ctx->prop_total;
  lc.refreshes = ctx->refreshes;
  lc.ties = ctx->ties;
  lc.cursor = ctx->opt_balance ? ctx->cursor : nullptr;
  lc.max_drift = ctx->max_drift;
  lc.ldet = ctx->ldet;
  lc.flags = ctx->flags;
  lc.acc_list = ctx->acc_list;
  lc.acc_cnt = ctx->acc_cnt;
  lc.scratch = ctx->scratch;
  lc.dly = 0;                      // set by record_sweep when the window is delayed
  lc.nidx = ctx->nidx;
  lc.dU = ctx->blk_U;
  lc.dr = ctx->blk_r;
  lc.dcnt = ctx->dly_cnt;
  lc.dBinv = ctx->blk_A;
  lc.dX = ctx->dly_dX;
  lc.dP = ctx->blk_D;
  lc.dP_off = ctx->blk_doff;
  lc.key0 = static_cast<uint32_t>(ctx->seed & 0xFFFFFFFFu);
  lc.key1 = static_cast<uint32_t>(ctx->seed >> 32);
  lc.n_chains = ctx->n_chains;
  lc.tile_kinds = ctx->tile_kinds;
  return lc;
}

int gj_nb(const ggf_ctx *ctx, int n_max) {
  // measured on the float64 matrix-core update: 256 wins from n = 2048 up, 128 at n = 512
  const int want = ctx->opt_gj_nb > 0 ? ctx->opt_gj_nb : (n_max >= 2048 ? 256 : n_max >= 512 ? 128 : 64);
  int nb = 8;
  while (nb < want && nb < 256) nb *= 2;   // power of two, 8..256
  return nb;
}

// Refactorise the listed chains from their link fields (float64 scratch, in chunks
// that fit the scratch budget), then recompute S for K > 1.  Synchronous.
ggf_status factorize(ggf_ctx *ctx, const std::vector<int> &which, int is_refresh, hipStream_t s) {
  if (which.empty()) return GGF_OK;
  size_t pos = 0;
  int all_nmax = 0;
  for (int c : which) all_nmax = std::max(all_nmax, ctx->chains[c].n);
  const int nb = gj_nb(ctx, all_nmax);
  while (pos < which.size()) {
    std::vector<int> chunk;
    size_t used = 0, yused = 0;
    int nmax = 0;
    while (pos < which.size()) {
      const int c = which[pos];
      const size_t need = static_cast<size_t>(ctx->chains[c].n) * ctx->chains[c].n;
      if (!chunk.empty() && used + need > ctx->scratch_elems) break;
      ctx->chains[c].scr_off = used;
      used += (need + 63) & ~static_cast<size_t>(63);
      ctx->chains[c].y_off = yused;
      yused += static_cast<size_t>(nb) * ctx->chains[c].n;
      nmax = std::max(nmax, ctx->chains[c].n);
      chunk.push_back(c);
      ++pos;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->chains_dev, ctx->chains.data(), ctx->chains.size() * sizeof(ChainDev),
                                hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->list_dev, chunk.data(), chunk.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const LaunchCtx lc = launch_ctx(ctx, s);
    const int cnt = static_cast<int>(chunk.size());
    ggf_launch_assemble(lc, ctx->list_dev, cnt, nmax / 8);
    if (yused > ctx->ybuf_elems) {
      if (ctx->ybuf) hipFree(ctx->ybuf);
      ctx->ybuf = nullptr;
      ctx->ybuf_elems = 0;
      HIP_TRY(ctx, hipMalloc(&ctx->ybuf, yused * sizeof(double)));
      ctx->ybuf_elems = yused;
    }
    ggf_launch_gj(lc, ctx->list_dev, cnt, nmax, nb, ctx->piv, ctx->perm, ctx->piv_stride, ctx->ybuf);
    ggf_launch_store(lc, ctx->list_dev, cnt, nmax, ctx->perm, ctx->piv_stride);
    ggf_launch_post(lc, ctx->list_dev, cnt, is_refresh);
    ggf_launch_sfac(lc, ctx->list_dev, cnt, ctx->kmax);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  std::vector<int> fl(ctx->n_chains);
  HIP_TRY(ctx, hipMemcpy(fl.data(), ctx->flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost));
  for (int c : which)
    if (fl[c] & GGF_FLAG_SINGULAR)
      return fail(ctx, GGF_ESINGULAR, "M(G) is singular (W(G) = 0) for chain " + std::to_string(c));
  return GGF_OK;
}

// Window length of delayed updates: the option, else 16 link steps (rank-64
// flushes), 0 = immediate rank-4 updates.  Multiples of 8 keep the partial last
// window of a sweep (2 L^2 link steps) at a rank that is a multiple of 32.
int delay_window(const ggf_ctx *ctx) {
  const int want = ctx->opt_delay >= 0 ? ctx->opt_delay : 16;
  return want;
}

ggf_status block_buffers(ggf_ctx *ctx);

// State of delayed updates: the block-move buffers (window inverse, W, pending
// Majoranas, operands of the window flush) plus the pending link changes and the
// window-list counters; independent of the window length.
ggf_status delay_buffers(ggf_ctx *ctx, int F) {
  if (F == 0 || ctx->dly_cnt) return GGF_OK;
  ggf_status st = block_buffers(ctx);
  if (st != GGF_OK) return st;
  hipError_t e = hipSuccess;
  ctx->dly_dX = dalloc<double>(ctx, static_cast<size_t>(GGF_BLOCK_RMAX) * ctx->n_chains, e);
  ctx->dly_cnt = dalloc<int>(ctx, 2, e);
  if (e != hipSuccess) return fail(ctx, GGF_ENOMEM, "cannot allocate delayed-update buffers");
  return GGF_OK;
}

ggf_status record_sweep(ggf_ctx *ctx, hipStream_t s, bool timed) {
  LaunchCtx lc = launch_ctx(ctx, s);
  const int tiles = ctx->opt_update_tiles > 0 ? ctx->opt_update_tiles : std::max(1, ctx->n_max / 16);
  const int grid = ctx->opt_update_grid > 0 ? ctx->opt_update_grid : 2048;
  const int F = delay_window(ctx);
  if (F > 0 && !ctx->dly_cnt) return fail(ctx, GGF_ESTATE, "delayed-update buffers are not allocated");
  // measured on the buffer-addressed flush: 512 workgroups beat 1024 by 2.5 % at 4096 chains of n = 128
  const int flush_grid = ctx->opt_flush_grid > 0 ? ctx->opt_flush_grid : 512;
  lc.dly = F;
  int k = 0;
  for (int ell = 0; ell < ctx->max_links; ++ell) {
    const int t = F > 0 ? ell % F : 0;
    const int wp = F > 0 ? (ell / F) & 1 : 0;
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->rev[2 * ell], s));
    ggf_launch_ratio(lc, ell, ell & 1, ctx->kmax, t, wp);
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->rev[2 * ell + 1], s));
    if (F > 0 && t != F - 1 && ell != ctx->max_links - 1) continue;
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2 * k], s));
    if (F > 0) ggf_launch_window_flush(lc, wp, flush_grid, ctx->kmax > 1);
    else ggf_launch_update(lc, ell & 1, grid, tiles, ctx->opt_update_nt);
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2 * k + 1], s));
    ++k;
  }
  ctx->timed_launches = timed ? k : 0;
  ggf_launch_end_sweep(lc);
  HIP_TRY(ctx, hipGetLastError());
  return GGF_OK;
}

ggf_status after_sweep(ggf_ctx *ctx, hipStream_t s) {
  // refresh (every refresh_every accepted flips) and recovery from non-finite ratios
  std::vector<uint32_t> since(ctx->n_chains);
  std::vector<int> fl(ctx->n_chains);
  HIP_TRY(ctx, hipMemcpyAsync(since.data(), ctx->acc_since, since.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(fl.data(), ctx->flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  std::vector<int> refresh, recover;
  for (int c = 0; c < ctx->n_chains; ++c) {
    if (fl[c] & GGF_FLAG_NONFINITE) {
      recover.push_back(c);
      if (ctx->recoveries[c] > 0 && fl[c] == GGF_FLAG_NONFINITE) {
        // already recovered once and failed again in the next sweep
      }
    } else if (ctx->refresh_every > 0 && since[c] >= static_cast<uint32_t>(ctx->refresh_every)) {
      refresh.push_back(c);
    }
  }
  if (!recover.empty()) {
    std::vector<int> zero(ctx->n_chains, 0);
    for (int c : recover) {
      ctx->recoveries[c] += 1;
      fl[c] = 0;
    }
    HIP_TRY(ctx, hipMemcpy(ctx->flags, fl.data(), fl.size() * sizeof(int), hipMemcpyHostToDevice));
    ggf_status st = factorize(ctx, recover, 0, s);
    if (st != GGF_OK) return st;
    HIP_TRY(ctx, hipMemcpy(fl.data(), ctx->flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (int c : recover)
      if (fl[c] & GGF_FLAG_NONFINITE)
        return fail(ctx, GGF_ENONFINITE, "non-finite weight persists after refactorisation, chain " + std::to_string(c));
  }
  return factorize(ctx, refresh, 1, s);
}

NNArgs nn_args(ggf_ctx *ctx) {
  NNArgs n;
  n.P = ctx->nn_P;
  n.wq = ctx->nn_wq;
  n.params = ctx->nn_p;
  n.chains = ctx->chains_dev;
  n.links = ctx->links;
  return n;
}

// All chains must be Z2 lattices tiled by P x P patches.
ggf_status nn_check_chains(ggf_ctx *ctx) {
  if (ctx->nn_P == 0) return fail(ctx, GGF_ESTATE, "ggf_nn_init has not been called");
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  for (const ChainDev &c : ctx->chains) {
    if (c.group != 2) return fail(ctx, GGF_EINVAL, "the learned block proposal is defined for Z2 chains");
    if (c.L % ctx->nn_P != 0) return fail(ctx, GGF_EINVAL, "lattice side is not a multiple of the patch side");
  }
  return GGF_OK;
}

ggf_status nn_examples(ggf_ctx *ctx, int32_t n, const int32_t *chain, const int32_t *patch) {
  if (n <= 0 || !chain || !patch) return fail(ctx, GGF_EINVAL, "examples are required");
  for (int e = 0; e < n; ++e) {
    if (chain[e] < 0 || chain[e] >= ctx->n_chains) return fail(ctx, GGF_EINVAL, "example chain out of range");
    const int npx = ctx->chains[chain[e]].L / ctx->nn_P;
    if (patch[e] < 0 || patch[e] >= npx * npx) return fail(ctx, GGF_EINVAL, "example patch out of range");
  }
  if (n > ctx->nn_cap) return fail(ctx, GGF_EINVAL, "too many examples (capacity 65536)");
  HIP_TRY(ctx, hipMemcpy(ctx->nn_ex_chain, chain, n * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->nn_ex_patch, patch, n * sizeof(int), hipMemcpyHostToDevice));
  return GGF_OK;
}

ggf_status block_buffers(ggf_ctx *ctx) {
  if (ctx->blk_A) return GGF_OK;
  hipError_t e = hipSuccess;
  const size_t esz = ctx->precision == 64 ? sizeof(double) : sizeof(float);
  std::vector<size_t> off(ctx->n_chains);
  size_t tot = 0;
  for (int c = 0; c < ctx->n_chains; ++c) {
    off[c] = tot;
    tot += static_cast<size_t>(GGF_BLOCK_RMAX) * ctx->chains[c].n;
  }
  const size_t rr = static_cast<size_t>(GGF_BLOCK_RMAX) * GGF_BLOCK_RMAX;
  ctx->blk_A = dalloc<double>(ctx, rr * ctx->n_chains, e);
  ctx->blk_W = dalloc<double>(ctx, rr * ctx->n_chains, e);
  ctx->blk_doff = dalloc<size_t>(ctx, ctx->n_chains, e);
  ctx->blk_U = dalloc<int>(ctx, static_cast<size_t>(GGF_BLOCK_RMAX) * ctx->n_chains, e);
  ctx->blk_r = dalloc<int>(ctx, ctx->n_chains, e);
  // proposed, accepted, links changed, updates of G
  ctx->blk_prop = dalloc<unsigned long long>(ctx, 4 * static_cast<size_t>(ctx->n_chains), e);
  ctx->blk_acc = ctx->blk_prop;
  const size_t er = static_cast<size_t>(GGF_BLOCK_RMAX + 4 * (GGF_KMAX_DEV - 1)) * GGF_BLOCK_RMAX;
  ctx->blk_E = dalloc<double>(ctx, er * ctx->n_chains, e);
  ctx->blk_F = dalloc<double>(ctx, er * ctx->n_chains, e);
  ctx->blk_Wn = dalloc<double>(ctx, rr * ctx->n_chains, e);
  ctx->blk_Un = dalloc<int>(ctx, static_cast<size_t>(GGF_BLOCK_RMAX) * ctx->n_chains, e);
  ctx->blk_rn = dalloc<int>(ctx, ctx->n_chains, e);
  ctx->blk_mode = dalloc<int>(ctx, ctx->n_chains, e);
  for (void **dst : {&ctx->blk_D}) {
    if (e != hipSuccess) break;
    void *p = nullptr;
    e = hipMalloc(&p, tot * esz);
    if (e == hipSuccess) {
      ctx->allocs.push_back(p);
      *dst = p;
    }
  }
  if (e != hipSuccess) return fail(ctx, GGF_ENOMEM, "cannot allocate block-move buffers");
  HIP_TRY(ctx, hipMemcpy(ctx->blk_doff, off.data(), off.size() * sizeof(size_t), hipMemcpyHostToDevice));
  return GGF_OK;
}

}  // namespace

extern "C" {

ggf_status ggf_create(ggf_ctx **out, int device) {
  if (!out) return GGF_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GGF_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return GGF_EDEVICE;
  ggf_ctx *ctx = new (std::nothrow) ggf_ctx();
  if (!ctx) return GGF_ENOMEM;
  ctx->device = device;
  // the staging array's address on this device, looked up once per device at set-up
  ctx->stage_err = ggf_stage_address(device, &ctx->stage);
  *out = ctx;
  return GGF_OK;
}

ggf_status ggf_set_tensor(ggf_ctx *ctx, const ggf_tensor_desc *d, int32_t *tensor_id_out) {
  if (!ctx) return GGF_EINVAL;
  if (!d || !tensor_id_out || !d->gamma_loc || !d->gamma_bond) return fail(ctx, GGF_EINVAL, "null descriptor field");
  if (d->group < 2 || d->group > GGF_ZN_MAX) return fail(ctx, GGF_EINVAL, "group must be in 2..64");
  if (d->K < 1 || d->K > GGF_KMAX) return fail(ctx, GGF_EINVAL, "K must be in 1..GGF_KMAX");
  if (d->K > 1 && (!d->patch_link || !d->gamma_bond_k || !d->c_re || !d->c_im))
    return fail(ctx, GGF_EINVAL, "K > 1 needs patch_link, gamma_bond_k, c_re, c_im");
  std::string why;
  if (!check_local(d->gamma_loc, why)) return fail(ctx, GGF_EINVAL, why);
  TensorDev t;
  std::memset(&t, 0, sizeof(t));
  t.group = d->group;
  t.K = d->K;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) t.a[i * 2 + j] = d->gamma_loc[i * 10 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 8; ++j) t.b[i * 8 + j] = d->gamma_loc[i * 10 + 2 + j];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) t.d[i * 8 + j] = d->gamma_loc[(2 + i) * 10 + 2 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) t.x0[i * 2 + j] = d->gamma_bond[i * 4 + 2 + j];
  // the reference bond only couples out to in
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      if (std::fabs(d->gamma_bond[i * 4 + j]) > 1e-12 || std::fabs(d->gamma_bond[(2 + i) * 4 + 2 + j]) > 1e-12)
        return fail(ctx, GGF_EINVAL, "reference bond must only couple the out and in modes");
  Even2 b0;
  if (!even_state(d->gamma_bond, b0, why)) return fail(ctx, GGF_EINVAL, "gamma_bond: " + why);
  const int K = d->K;
  std::vector<Even2> bk(K);
  std::vector<cplx> cc(K, 1.0);
  bk[0] = b0;
  for (int k = 1; k < K; ++k) {
    if (!even_state(d->gamma_bond_k + 16 * k, bk[k], why))
      return fail(ctx, GGF_EINVAL, "gamma_bond_k[" + std::to_string(k) + "]: " + why);
    const cplx ov = std::conj(b0.a) * bk[k].a + std::conj(b0.b) * bk[k].b;   // <b_0|b_k>
    if (std::abs(ov) < 1e-12) return fail(ctx, GGF_EINVAL, "<b_0|b_k> = 0: phase convention undefined");
    const cplx ph = ov / std::abs(ov);
    bk[k].a /= ph;
    bk[k].b /= ph;
    if (d->patch_link[k] < 0) return fail(ctx, GGF_EINVAL, "patch_link[k] must be >= 0 for k >= 1");
  }
  if (K > 1)
    for (int k = 0; k < K; ++k) cc[k] = cplx(d->c_re[k], d->c_im[k]);
  HostBonds hb;
  hb.bk = bk;
  hb.cc = cc;
  hb.patch.assign(d->patch_link ? d->patch_link : nullptr, d->patch_link ? d->patch_link + K : nullptr);
  if (hb.patch.empty()) hb.patch.assign(K, -1);
  for (int q = 0; q < 16; ++q) hb.g0[q] = d->gamma_bond[q];
  if (!fill_pairs(t, hb, why)) return fail(ctx, GGF_EINVAL, why);
  ctx->bonds.push_back(hb);
  ctx->tensors.push_back(t);
  if (ctx->tensors.size() > ctx->tensors_cap) {
    // a captured sweep graph holds the old table's address in its kernel arguments
    if (ctx->graph_exec) { hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
    if (ctx->tensors_dev) hipFree(ctx->tensors_dev);
    ctx->tensors_cap = std::max<size_t>(16, 2 * ctx->tensors.size());
    HIP_TRY(ctx, hipMalloc(&ctx->tensors_dev, ctx->tensors_cap * sizeof(TensorDev)));
  }
  HIP_TRY(ctx, hipMemcpy(ctx->tensors_dev, ctx->tensors.data(), ctx->tensors.size() * sizeof(TensorDev),
                         hipMemcpyHostToDevice));
  *tensor_id_out = static_cast<int32_t>(ctx->tensors.size() - 1);
  return GGF_OK;
}

ggf_status ggf_init_chains(ggf_ctx *ctx, int32_t n_chains, const int32_t *L, const int32_t *tensor_id,
                           uint64_t seed, int32_t init, int32_t precision, int32_t refresh_every, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (n_chains <= 0 || !L || !tensor_id) return fail(ctx, GGF_EINVAL, "n_chains, L and tensor_id are required");
  if (precision != 32 && precision != 64) return fail(ctx, GGF_EINVAL, "precision must be 32 or 64");
  if (init != 0 && init != 1) return fail(ctx, GGF_EINVAL, "init must be 0 (cold) or 1 (hot)");
  if (refresh_every < 0) return fail(ctx, GGF_EINVAL, "refresh_every must be >= 0");
  std::vector<ChainDev> ch(n_chains);
  size_t goff = 0, foff = 0, loff = 0;
  int kmax = 1, max_links = 0, n_max = 0, nidx = 4;
  size_t max_need = 0, tot_need = 0;
  for (int c = 0; c < n_chains; ++c) {
    const int l = L[c];
    if (l < 2 || l > 32 || (l & 1)) return fail(ctx, GGF_EINVAL, "L must be even and in 2..32");
    const int tid = tensor_id[c];
    if (tid < 0 || tid >= static_cast<int>(ctx->tensors.size())) return fail(ctx, GGF_EINVAL, "bad tensor id");
    const TensorDev &t = ctx->tensors[tid];
    for (int n = 0; n < t.K; ++n)
      for (int m = 0; m < t.K; ++m)
        for (int q = 0; q < t.nl[n][m]; ++q)
          if (t.lk[n][m][q] >= 2 * l * l) return fail(ctx, GGF_EINVAL, "patch link outside the lattice");
    ChainDev &d = ch[c];
    std::memset(&d, 0, sizeof(d));
    d.L = l;
    d.n = 8 * l * l;
    d.nlinks = 2 * l * l;
    d.tensor = tid;
    d.group = t.group;
    d.K = t.K;
    d.g_off = goff;
    d.f_off = foff;
    d.link_off = loff;
    const size_t nn = static_cast<size_t>(d.n) * d.n;
    goff += (nn + 63) & ~static_cast<size_t>(63);
    foff += 8 * static_cast<size_t>(d.n);
    loff += (d.nlinks + 63) & ~63;
    kmax = std::max(kmax, t.K);
    {
      // index set of a link step: U plus the Majoranas of every distinct patch link of the pairs
      std::vector<int> pl;
      for (int a = 0; a < t.K; ++a)
        for (int b = a; b < t.K; ++b)
          if (a + b > 0)
            for (int l = 0; l < t.nl[a][b]; ++l)
              if (std::find(pl.begin(), pl.end(), t.lk[a][b][l]) == pl.end()) pl.push_back(t.lk[a][b][l]);
      nidx = std::max(nidx, std::min(16, 4 + 4 * static_cast<int>(pl.size())));
    }
    max_links = std::max(max_links, d.nlinks);
    n_max = std::max(n_max, d.n);
    max_need = std::max(max_need, nn);
    tot_need += (nn + 63) & ~static_cast<size_t>(63);
  }
  free_chains(ctx);
  hipError_t e = hipSuccess;
  const size_t esz = precision == 64 ? sizeof(double) : sizeof(float);
  size_t scr = tot_need;
  const size_t budget = ctx->opt_scratch_mb > 0 ? static_cast<size_t>(ctx->opt_scratch_mb) << 20
                                                : (static_cast<size_t>(32) << 30);
  scr = std::min(scr, std::max(budget / sizeof(double), max_need));
  {
    void *p = nullptr;
    e = hipMalloc(&p, goff * esz);
    if (e != hipSuccess) return fail(ctx, GGF_ENOMEM, "cannot allocate the inverse arena");
    ctx->allocs.push_back(p);
    ctx->G = p;
    e = hipMalloc(&p, foff * esz);
    if (e != hipSuccess) { free_chains(ctx); return fail(ctx, GGF_ENOMEM, "cannot allocate the factor arena"); }
    ctx->allocs.push_back(p);
    ctx->F = p;
    e = hipMalloc(&p, scr * sizeof(double));
    if (e != hipSuccess) { free_chains(ctx); return fail(ctx, GGF_ENOMEM, "cannot allocate the refactorisation scratch"); }
    ctx->allocs.push_back(p);
    ctx->scratch = static_cast<double *>(p);
    ctx->scratch_elems = scr;
  }
  ctx->links = dalloc<int8_t>(ctx, loff, e);
  ctx->logw = dalloc<double>(ctx, n_chains, e);
  ctx->max_drift = dalloc<double>(ctx, n_chains, e);
  ctx->ldet = dalloc<double>(ctx, n_chains, e);
  ctx->sfac = dalloc<double2>(ctx, n_chains, e);
  ctx->sweep = dalloc<uint32_t>(ctx, n_chains, e);
  ctx->acc_since = dalloc<uint32_t>(ctx, n_chains, e);
  ctx->acc_total = dalloc<unsigned long long>(ctx, n_chains, e);
  ctx->prop_total = dalloc<unsigned long long>(ctx, n_chains, e);
  ctx->refreshes = dalloc<unsigned long long>(ctx, n_chains, e);
  ctx->ties = dalloc<unsigned long long>(ctx, n_chains, e);
  ctx->cursor = dalloc<int>(ctx, n_chains, e);
  ctx->flags = dalloc<int>(ctx, n_chains, e);
  ctx->acc_list = dalloc<int>(ctx, n_chains, e);
  ctx->acc_cnt = dalloc<int>(ctx, 2, e);
  ctx->piv_stride = n_max;
  ctx->piv = dalloc<int>(ctx, static_cast<size_t>(n_chains) * n_max, e);
  ctx->perm = dalloc<int>(ctx, static_cast<size_t>(n_chains) * n_max, e);
  ctx->list_dev = dalloc<int>(ctx, n_chains, e);
  ctx->chains_dev = dalloc<ChainDev>(ctx, n_chains, e);
  if (e != hipSuccess) { free_chains(ctx); return fail(ctx, GGF_ENOMEM, "device allocation failed"); }
  ctx->chains = ch;
  ctx->n_chains = n_chains;
  ctx->precision = precision;
  ctx->refresh_every = refresh_every;
  ctx->kmax = kmax;
  ctx->nidx = nidx;
  ctx->tile_kinds = 0;
  for (const ChainDev &c : ch) ctx->tile_kinds |= c.n % GGF_WINDOW_TILE == 0 ? 1 : 2;
  ctx->max_links = max_links;
  ctx->n_max = n_max;
  ctx->seed = seed;
  ctx->recoveries.assign(n_chains, 0);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipMemcpy(ctx->chains_dev, ch.data(), ch.size() * sizeof(ChainDev), hipMemcpyHostToDevice));
  if (init == 1) {
    ggf_launch_hot_start(launch_ctx(ctx, s), max_links);
    HIP_TRY(ctx, hipGetLastError());
  }
  std::vector<int> all(n_chains);
  for (int c = 0; c < n_chains; ++c) all[c] = c;
  return factorize(ctx, all, 0, s);
}

ggf_status ggf_sweep(ggf_ctx *ctx, int32_t n_sweeps, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (n_sweeps < 0) return fail(ctx, GGF_EINVAL, "n_sweeps must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ggf_status dst = delay_buffers(ctx, delay_window(ctx));
  if (dst != GGF_OK) return dst;
  const bool timed = ctx->opt_time_update != 0;
  ctx->last_update_ms = 0.0;
  ctx->last_launches = 0;
  ctx->last_flips = 0;
  ctx->last_ratio_ms = 0.0;
  ctx->last_ratio_launches = 0;
  if (timed && (ctx->tev.size() < static_cast<size_t>(2 * ctx->max_links) ||
                ctx->rev.size() < static_cast<size_t>(2 * ctx->max_links))) {
    for (hipEvent_t ev : ctx->tev) hipEventDestroy(ev);
    for (hipEvent_t ev : ctx->rev) hipEventDestroy(ev);
    ctx->tev.assign(2 * ctx->max_links, nullptr);
    ctx->rev.assign(2 * ctx->max_links, nullptr);
    for (auto &ev : ctx->tev) HIP_TRY(ctx, hipEventCreate(&ev));
    for (auto &ev : ctx->rev) HIP_TRY(ctx, hipEventCreate(&ev));
  }
  std::vector<unsigned long long> acc0;
  if (timed) {
    acc0.resize(ctx->n_chains);
    HIP_TRY(ctx, hipMemcpy(acc0.data(), ctx->acc_total, acc0.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  }
  for (int sw = 0; sw < n_sweeps; ++sw) {
    if (ctx->opt_graph && !timed) {
      if (!ctx->own_stream) {
        HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
      }
      if (!ctx->graph_exec) {
        hipGraph_t g;
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->own_stream, hipStreamCaptureModeThreadLocal));
        ggf_status st = record_sweep(ctx, ctx->own_stream, false);
        hipError_t e = hipStreamEndCapture(ctx->own_stream, &g);
        if (st != GGF_OK) return st;
        if (e != hipSuccess) return fail(ctx, GGF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        HIP_TRY(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
        hipGraphDestroy(g);
      }
      HIP_TRY(ctx, hipEventRecord(ctx->ev_in, s));
      HIP_TRY(ctx, hipStreamWaitEvent(ctx->own_stream, ctx->ev_in, 0));
      HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->own_stream));
      HIP_TRY(ctx, hipEventRecord(ctx->ev_out, ctx->own_stream));
      HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->ev_out, 0));
    } else {
      ggf_status st = record_sweep(ctx, s, timed);
      if (st != GGF_OK) return st;
      if (timed) {
        HIP_TRY(ctx, hipStreamSynchronize(s));
        for (int k = 0; k < ctx->timed_launches; ++k) {
          float ms = 0.f;
          HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->tev[2 * k], ctx->tev[2 * k + 1]));
          ctx->last_update_ms += ms;
        }
        ctx->last_launches += ctx->timed_launches;
        for (int ell = 0; ell < ctx->max_links; ++ell) {
          float ms = 0.f;
          HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->rev[2 * ell], ctx->rev[2 * ell + 1]));
          ctx->last_ratio_ms += ms;
        }
        ctx->last_ratio_launches += ctx->max_links;
      }
    }
    ggf_status st = after_sweep(ctx, s);
    if (st != GGF_OK) return st;
  }
  if (timed) {
    std::vector<unsigned long long> acc1(ctx->n_chains);
    HIP_TRY(ctx, hipMemcpy(acc1.data(), ctx->acc_total, acc1.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (int c = 0; c < ctx->n_chains; ++c) ctx->last_flips += static_cast<long long>(acc1[c] - acc0[c]);
  }
  return GGF_OK;
}

ggf_status ggf_measure(ggf_ctx *ctx, uint32_t obs_mask, double *out, int32_t out_is_device, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (!out) return fail(ctx, GGF_EINVAL, "out is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LaunchCtx lc = launch_ctx(ctx, s);
  const size_t bytes = static_cast<size_t>(ctx->n_chains) * GGF_NOBS * sizeof(double);
  if (out_is_device) {
    ggf_launch_measure(lc, obs_mask, out, ctx->kmax);
    HIP_TRY(ctx, hipGetLastError());
    return GGF_OK;
  }
  double *tmp = nullptr;
  HIP_TRY(ctx, hipMalloc(&tmp, bytes));
  ggf_launch_measure(lc, obs_mask, tmp, ctx->kmax);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(tmp);
  if (e != hipSuccess) return fail(ctx, GGF_EDEVICE, std::string("measure: ") + hipGetErrorString(e));
  return GGF_OK;
}

ggf_status ggf_measure_staged(ggf_ctx *ctx, uint32_t obs_mask, double *host_out, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (!host_out) return fail(ctx, GGF_EINVAL, "host_out is NULL");
  if (ctx->n_chains > GGF_STAGE_MAX_CHAINS)
    return fail(ctx, GGF_EINVAL, "ggf_measure_staged stages at most " + std::to_string(GGF_STAGE_MAX_CHAINS) +
                                     " chains, the context has " + std::to_string(ctx->n_chains));
  if (!ctx->stage)
    return fail(ctx, GGF_EDEVICE, std::string("staging array unavailable: ") + hipGetErrorString(ctx->stage_err));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LaunchCtx lc = launch_ctx(ctx, s);
  // every slot of every row is written by the measurement, so the array needs no clearing
  ggf_launch_measure(lc, obs_mask, ctx->stage, ctx->kmax);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipMemcpyAsync(host_out, ctx->stage, static_cast<size_t>(ctx->n_chains) * GGF_NOBS * sizeof(double),
                              hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return GGF_OK;
}

ggf_status ggf_set_lambda(ggf_ctx *ctx, int32_t tensor_id, const double *c_re, const double *c_im, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (tensor_id < 0 || tensor_id >= static_cast<int32_t>(ctx->tensors.size()))
    return fail(ctx, GGF_EINVAL, "bad tensor id");
  if (!c_re || !c_im) return fail(ctx, GGF_EINVAL, "c_re and c_im are required");
  TensorDev &t = ctx->tensors[tensor_id];
  const int K = t.K;
  if (K == 1) return GGF_OK;   // a single Gaussian: lambda only scales the state
  double nrm = 0.0;
  for (int k = 0; k < K; ++k) {
    if (!std::isfinite(c_re[k]) || !std::isfinite(c_im[k])) return fail(ctx, GGF_EINVAL, "lambda must be finite");
    nrm += c_re[k] * c_re[k] + c_im[k] * c_im[k];
  }
  if (!(nrm > 0.0)) return fail(ctx, GGF_EINVAL, "lambda must not vanish");
  for (int n = 0; n < K; ++n)
    for (int m = 0; m < K; ++m) {
      const cplx w = std::conj(cplx(c_re[n], c_im[n])) * cplx(c_re[m], c_im[m]) *
                     cplx(t.ov[n][m].x, t.ov[n][m].y);
      t.w[n][m] = make_double2(w.real(), w.imag());
    }
  for (int k = 0; k < K; ++k) ctx->bonds[tensor_id].cc[k] = cplx(c_re[k], c_im[k]);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->tensors_dev + tensor_id, &t, sizeof(TensorDev), hipMemcpyHostToDevice, s));
  std::vector<int> which;
  for (int c = 0; c < ctx->n_chains; ++c)
    if (ctx->chains[c].tensor == tensor_id) which.push_back(c);
  if (!which.empty()) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->list_dev, which.data(), which.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const LaunchCtx lc = launch_ctx(ctx, s);
    ggf_launch_sfac(lc, ctx->list_dev, static_cast<int>(which.size()), ctx->kmax);
    HIP_TRY(ctx, hipGetLastError());
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return GGF_OK;
}

ggf_status ggf_set_bond(ggf_ctx *ctx, int32_t tensor_id, int32_t k, const double *gamma_bond_k, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (tensor_id < 0 || tensor_id >= static_cast<int32_t>(ctx->tensors.size()))
    return fail(ctx, GGF_EINVAL, "bad tensor id");
  TensorDev &t = ctx->tensors[tensor_id];
  if (k < 1 || k >= t.K) return fail(ctx, GGF_EINVAL, "k must be in 1 .. K - 1");
  if (!gamma_bond_k) return fail(ctx, GGF_EINVAL, "gamma_bond_k is required");
  std::string why;
  Even2 b;
  if (!even_state(gamma_bond_k, b, why)) return fail(ctx, GGF_EINVAL, "gamma_bond_k: " + why);
  HostBonds hb = ctx->bonds[tensor_id];
  const cplx ov = std::conj(hb.bk[0].a) * b.a + std::conj(hb.bk[0].b) * b.b;
  if (std::abs(ov) < 1e-12) return fail(ctx, GGF_EINVAL, "<b_0|b_k> = 0: phase convention undefined");
  const cplx ph = ov / std::abs(ov);
  b.a /= ph;
  b.b /= ph;
  hb.bk[k] = b;
  TensorDev nt = t;
  if (!fill_pairs(nt, hb, why)) return fail(ctx, GGF_EINVAL, why);
  t = nt;
  ctx->bonds[tensor_id] = hb;
  // G = M_00^-1 and W(G) do not involve the patch bonds; only S(G) = N(G) / W(G) changes
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->tensors_dev + tensor_id, &t, sizeof(TensorDev), hipMemcpyHostToDevice, s));
  std::vector<int> which;
  for (int c = 0; c < ctx->n_chains; ++c)
    if (ctx->chains[c].tensor == tensor_id) which.push_back(c);
  if (!which.empty()) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->list_dev, which.data(), which.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const LaunchCtx lc = launch_ctx(ctx, s);
    ggf_launch_sfac(lc, ctx->list_dev, static_cast<int>(which.size()), ctx->kmax);
    HIP_TRY(ctx, hipGetLastError());
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return GGF_OK;
}

ggf_status ggf_measure_energy(ggf_ctx *ctx, const ggf_couplings *cp, double *out, int32_t out_is_device,
                              void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (!out || !cp) return fail(ctx, GGF_EINVAL, "out and couplings are required");
  const double cv[5] = {cp->t, cp->mu, cp->m, cp->kb, cp->ke};
  for (double v : cv)
    if (!std::isfinite(v)) return fail(ctx, GGF_EINVAL, "couplings must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LaunchCtx lc = launch_ctx(ctx, s);
  const EnergyCp ec{cp->t, cp->mu, cp->m, cp->kb, cp->ke};
  const size_t bytes = static_cast<size_t>(ctx->n_chains) * GGF_ENERGY_STRIDE * sizeof(double);
  if (out_is_device) {
    ggf_launch_energy(lc, ec, out, ctx->kmax);
    HIP_TRY(ctx, hipGetLastError());
    return GGF_OK;
  }
  double *tmp = nullptr;
  HIP_TRY(ctx, hipMalloc(&tmp, bytes));
  ggf_launch_energy(lc, ec, tmp, ctx->kmax);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(tmp);
  if (e != hipSuccess) return fail(ctx, GGF_EDEVICE, std::string("measure_energy: ") + hipGetErrorString(e));
  return GGF_OK;
}

ggf_status ggf_measure_bond_rows(ggf_ctx *ctx, const ggf_couplings *cp, double *out, int32_t out_is_device,
                                 void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (!out || !cp) return fail(ctx, GGF_EINVAL, "out and couplings are required");
  const double cv[5] = {cp->t, cp->mu, cp->m, cp->kb, cp->ke};
  for (double v : cv)
    if (!std::isfinite(v)) return fail(ctx, GGF_EINVAL, "couplings must be finite");
  for (const ChainDev &ch : ctx->chains) {
    if (ch.K < 2) continue;
    const TensorDev &t = ctx->tensors[ch.tensor];
    std::vector<int> S;
    for (int k = 1; k < ch.K; ++k) {
      const int ell = t.lk[k][0][0], i = ell >> 1, mu = ell & 1, L = ch.L;
      const int j = mu == 0 ? (i / L) * L + (i % L + 1) % L : ((i / L + 1) % L) * L + i % L;
      const int u[4] = {mu == 0 ? 8 * i + 4 : 8 * i + 2, mu == 0 ? 8 * i + 5 : 8 * i + 3,
                        mu == 0 ? 8 * j + 0 : 8 * j + 6, mu == 0 ? 8 * j + 1 : 8 * j + 7};
      for (int q : u)
        if (std::find(S.begin(), S.end(), q) == S.end()) S.push_back(q);
    }
    if (static_cast<int>(S.size()) * ch.L * ch.L > 4096)
      return fail(ctx, GGF_EINVAL, "bond rows need s L^2 <= 4096 (s = 4 (K - 1) patch Majoranas)");
  }
  static_assert(GGF_BOND_STRIDE == GGF_BOND_STRIDE_DEV, "row size");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LaunchCtx lc = launch_ctx(ctx, s);
  const EnergyCp ec{cp->t, cp->mu, cp->m, cp->kb, cp->ke};
  if (out_is_device) {
    ggf_launch_bond_rows(lc, ec, out);
    HIP_TRY(ctx, hipGetLastError());
    return GGF_OK;
  }
  const size_t bytes = static_cast<size_t>(ctx->n_chains) * GGF_BOND_STRIDE * sizeof(double);
  double *tmp = nullptr;
  HIP_TRY(ctx, hipMalloc(&tmp, bytes));
  ggf_launch_bond_rows(lc, ec, tmp);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(tmp);
  if (e != hipSuccess) return fail(ctx, GGF_EDEVICE, std::string("measure_bond_rows: ") + hipGetErrorString(e));
  return GGF_OK;
}

namespace {

// ----- gradient with respect to the patch bond states (host) -----
// Derivative of a bond state a|00> + b|11> along Gamma -> exp(theta E) Gamma exp(-theta E): the
// state is the ground state of the even-sector H = [[h, z], [z^*, -h]] (even_state), so first-order
// perturbation theory in that 2 x 2 block is exact: dv = -w <w|dH|v> / (2 e), w = (-b^*, a^*) the
// excited state, e = sqrt(h^2 + |z|^2), dH from dGamma = [E, Gamma] by the same linear map; then the
// phase convention <b_0|b_k> > 0 adds -i Im(<b_0|dv> / <b_0|v>) v.
Even2 bond_state_derivative(const double *g, const double *E, const Even2 &v, const Even2 &b0) {
  double dg[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double x = 0.0;
      for (int q = 0; q < 4; ++q) x += E[i * 4 + q] * g[q * 4 + j] - g[i * 4 + q] * E[q * 4 + j];
      dg[i * 4 + j] = x;
    }
  const double h = 0.5 * (g[0 * 4 + 1] + g[2 * 4 + 3]);
  const cplx z(0.5 * (g[0 * 4 + 3] + g[1 * 4 + 2]), 0.5 * (g[0 * 4 + 2] - g[1 * 4 + 3]));
  const double dh = 0.5 * (dg[0 * 4 + 1] + dg[2 * 4 + 3]);
  const cplx dz(0.5 * (dg[0 * 4 + 3] + dg[1 * 4 + 2]), 0.5 * (dg[0 * 4 + 2] - dg[1 * 4 + 3]));
  const double e = std::sqrt(h * h + std::norm(z));
  const cplx wa = -std::conj(v.b), wb = std::conj(v.a);
  // dH v and <w|dH v>
  const cplx hva = dh * v.a + dz * v.b, hvb = std::conj(dz) * v.a - dh * v.b;
  const cplx amp = std::conj(wa) * hva + std::conj(wb) * hvb;
  Even2 dv{-wa * amp / (2.0 * e), -wb * amp / (2.0 * e)};
  const cplx ov = std::conj(b0.a) * v.a + std::conj(b0.b) * v.b;
  const cplx dov = std::conj(b0.a) * dv.a + std::conj(b0.b) * dv.b;
  const cplx ph(0.0, -std::imag(dov / ov));
  dv.a += ph * v.a;
  dv.b += ph * v.b;
  return dv;
}

// Derivatives of a link's transition quantities (transition_cov, occupation_response and the
// overlap <bra|ket>) for bond vectors moving by (dbra, dket).
void transition_derivative(const Even2 &bra, const Even2 &ket, const Even2 &dbra, const Even2 &dket, cplx dg[16],
                           cplx &dov, cplx &den, cplx deq[16]) {
  const cplx ov = std::conj(bra.a) * ket.a + std::conj(bra.b) * ket.b;
  dov = std::conj(dbra.a) * ket.a + std::conj(dbra.b) * ket.b + std::conj(bra.a) * dket.a + std::conj(bra.b) * dket.b;
  cplx g[16], nb, q[16];
  transition_cov(bra, ket, g);
  occupation_response(bra, ket, nb, q);
  den = (std::conj(dbra.b) * ket.b + std::conj(bra.b) * dket.b) / ov - nb * dov / ov;
  for (int i = 0; i < 16; ++i) dg[i] = deq[i] = 0.0;
  for (int p = 0; p < 4; ++p)
    for (int r = p + 1; r < 4; ++r) {
      cplx m[2][2];
      bilinear(p, r, m);
      auto mel = [&](const Even2 &x, const Even2 &y) {
        return std::conj(x.a) * (m[0][0] * y.a + m[0][1] * y.b) + std::conj(x.b) * (m[1][0] * y.a + m[1][1] * y.b);
      };
      const cplx e = mel(bra, ket), de = mel(dbra, ket) + mel(bra, dket);
      const cplx I(0.0, 1.0);
      const cplx dgv = I * de / ov - I * e * dov / (ov * ov);
      // Q_pr = i <bra|n_out c_p c_r|ket> / ov - Gamma_pr nbar, n_out = |11><11|
      const cplx e1 = std::conj(bra.b) * (m[1][0] * ket.a + m[1][1] * ket.b);
      const cplx de1 = std::conj(dbra.b) * (m[1][0] * ket.a + m[1][1] * ket.b) +
                       std::conj(bra.b) * (m[1][0] * dket.a + m[1][1] * dket.b);
      const cplx dqv = I * de1 / ov - I * e1 * dov / (ov * ov) - dgv * nb - g[p * 4 + r] * den;
      dg[p * 4 + r] = dgv;
      dg[r * 4 + p] = -dgv;
      deq[p * 4 + r] = dqv;
      deq[r * 4 + p] = -dqv;
    }
}

// O X O^T for the link rotation O of value k (the out pair turned by 2 pi k / N).
void rotate4(const cplx x[16], int k, int group, cplx y[16]) {
  double c = 1.0, s = 0.0;
  if (k != 0) {
    if (group == 2) { c = -1.0; s = 0.0; }
    else { c = std::cos(2.0 * M_PI * k / group); s = std::sin(2.0 * M_PI * k / group); }
  }
  const double o[16] = {c, s, 0, 0, -s, c, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  cplx t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx v = 0.0;
      for (int q = 0; q < 4; ++q) v += o[i * 4 + q] * x[q * 4 + j];
      t[i * 4 + j] = v;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx v = 0.0;
      for (int q = 0; q < 4; ++q) v += t[i * 4 + q] * o[j * 4 + q];
      y[i * 4 + j] = v;
    }
}

// In-place inverse of an m x m complex matrix (m <= 8, leading dimension m) by Gauss-Jordan with
// partial pivoting; false when singular.
bool cinvert(std::vector<cplx> &a, int m) {
  std::vector<cplx> inv(m * m, 0.0);
  for (int i = 0; i < m; ++i) inv[i * m + i] = 1.0;
  for (int col = 0; col < m; ++col) {
    int p = col;
    for (int r = col + 1; r < m; ++r)
      if (std::abs(a[r * m + col]) > std::abs(a[p * m + col])) p = r;
    if (!(std::abs(a[p * m + col]) > 0.0)) return false;
    if (p != col)
      for (int j = 0; j < m; ++j) {
        std::swap(a[p * m + j], a[col * m + j]);
        std::swap(inv[p * m + j], inv[col * m + j]);
      }
    const cplx d = 1.0 / a[col * m + col];
    for (int j = 0; j < m; ++j) {
      a[col * m + j] *= d;
      inv[col * m + j] *= d;
    }
    for (int r = 0; r < m; ++r)
      if (r != col) {
        const cplx f = a[r * m + col];
        if (f == 0.0) continue;
        for (int j = 0; j < m; ++j) {
          a[r * m + j] -= f * a[col * m + j];
          inv[r * m + j] -= f * inv[col * m + j];
        }
      }
  }
  a = inv;
  return true;
}

}  // namespace

ggf_status ggf_bond_gradient(ggf_ctx *ctx, const ggf_tensor_desc *d, const ggf_couplings *cp,
                             const double *energy_rows, const double *bond_rows, int64_t n_rows, double *grad) {
  if (!d || !cp || !energy_rows || !bond_rows || n_rows <= 0 || !grad)
    return fail(ctx, GGF_EINVAL, "tensor, couplings, rows, n_rows > 0 and grad are required");
  const int K = d->K, group = d->group;
  if (K < 2 || K > GGF_KMAX || !d->patch_link || !d->gamma_bond_k || !d->c_re || !d->c_im)
    return fail(ctx, GGF_EINVAL, "the bond gradient needs a superposition (2 <= K <= GGF_KMAX) with its bonds");
  std::string why;
  std::vector<Even2> bk(K);
  if (!even_state(d->gamma_bond, bk[0], why)) return fail(ctx, GGF_EINVAL, "gamma_bond: " + why);
  for (int k = 1; k < K; ++k) {
    if (!even_state(d->gamma_bond_k + 16 * k, bk[k], why))
      return fail(ctx, GGF_EINVAL, "gamma_bond_k[" + std::to_string(k) + "]: " + why);
    const cplx ov = std::conj(bk[0].a) * bk[k].a + std::conj(bk[0].b) * bk[k].b;
    if (std::abs(ov) < 1e-12) return fail(ctx, GGF_EINVAL, "<b_0|b_k> = 0: phase convention undefined");
    const cplx ph = ov / std::abs(ov);
    bk[k].a /= ph;
    bk[k].b /= ph;
  }
  std::vector<cplx> cc(K);
  for (int k = 0; k < K; ++k) cc[k] = cplx(d->c_re[k], d->c_im[k]);
  const int ng = 6, gens[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  const int nout = (K - 1) * ng;
  // per-link transition data of pair (n, m): bra/ket bond vectors
  auto vectors = [&](int ell, int n, int m, Even2 &ket, Even2 &bra) {
    ket = (n > 0 && d->patch_link[n] == ell) ? bk[n] : bk[0];
    bra = (m > 0 && d->patch_link[m] == ell) ? bk[m] : bk[0];
  };
  cplx g0c[16];
  for (int i = 0; i < 16; ++i) g0c[i] = d->gamma_bond[i];
  cplx en0, eq0[16];
  occupation_response(bk[0], bk[0], en0, eq0);
  // bond derivatives per (k, generator)
  std::vector<Even2> dbk(nout);
  for (int k = 1; k < K; ++k)
    for (int gi = 0; gi < ng; ++gi) {
      double E[16] = {0.0};
      E[gens[gi][0] * 4 + gens[gi][1]] = 1.0;
      E[gens[gi][1] * 4 + gens[gi][0]] = -1.0;
      dbk[(k - 1) * ng + gi] = bond_state_derivative(d->gamma_bond_k + 16 * k, E, bk[k], bk[0]);
    }
  std::vector<double> es(n_rows), de(static_cast<size_t>(n_rows) * nout), dn(static_cast<size_t>(n_rows) * nout);
  for (int64_t r = 0; r < n_rows; ++r) {
    const double *er = energy_rows + r * GGF_ENERGY_STRIDE;
    const double *br = bond_rows + r * GGF_BOND_STRIDE;
    const int s = static_cast<int>(br[0]), L = static_cast<int>(br[1]);
    if (s < 4 || s > GGF_BOND_SMAX) return fail(ctx, GGF_EINVAL, "bond row " + std::to_string(r) + " has no patch set");
    std::vector<int> S(s);
    for (int q = 0; q < s; ++q) S[q] = static_cast<int>(br[2 + q]);
    auto link_pos = [&](int ell, int pos[4]) {
      const int i = ell >> 1, mu = ell & 1;
      const int j = mu == 0 ? (i / L) * L + (i % L + 1) % L : ((i / L + 1) % L) * L + i % L;
      const int u[4] = {mu == 0 ? 8 * i + 4 : 8 * i + 2, mu == 0 ? 8 * i + 5 : 8 * i + 3,
                        mu == 0 ? 8 * j + 0 : 8 * j + 6, mu == 0 ? 8 * j + 1 : 8 * j + 7};
      for (int q = 0; q < 4; ++q) pos[q] = static_cast<int>(std::find(S.begin(), S.end(), u[q]) - S.begin());
    };
    auto R = [&](int a, int b) { return cplx(br[18 + 2 * (12 * a + b)], br[19 + 2 * (12 * a + b)]); };
    auto gss = [&](int a, int b) { return br[306 + 12 * a + b]; };
    // pair weights and energies
    std::vector<cplx> om(K * K), h(K * K);
    cplx e = 0.0, Ssum = 0.0;
    for (int p = 0; p < K * K; ++p) {
      const cplx rs(er[1 + 4 * p], er[2 + 4 * p]), rhs(er[3 + 4 * p], er[4 + 4 * p]);
      om[p] = std::conj(cc[p / K]) * cc[p % K] * rs;   // om / S
      h[p] = rhs / rs;
      Ssum += om[p];
      e += om[p] * h[p];
    }
    es[r] = e.real();
    for (int k = 1; k < K; ++k) {
      const int ellk = d->patch_link[k];
      const int kv = static_cast<int>(br[14 + k]);
      int uk[4];
      link_pos(ellk, uk);
      for (int gi = 0; gi < ng; ++gi) {
        const Even2 &db = dbk[(k - 1) * ng + gi];
        cplx dE = 0.0, dN = 0.0;
        for (int n = 0; n < K; ++n)
          for (int m = 0; m < K; ++m) {
            if (n != k && m != k) continue;
            const int p = n * K + m;
            // the pair's patch links and their positions in S
            int links[2], nl = 0;
            if (n > 0) links[nl++] = d->patch_link[n];
            if (m > 0 && !(nl == 1 && links[0] == d->patch_link[m])) links[nl++] = d->patch_link[m];
            std::vector<int> P;
            std::vector<int> lpos(nl * 4);
            for (int l = 0; l < nl; ++l) {
              int pos[4];
              link_pos(links[l], pos);
              for (int q = 0; q < 4; ++q) {
                auto it = std::find(P.begin(), P.end(), pos[q]);
                if (it == P.end()) { lpos[l * 4 + q] = static_cast<int>(P.size()); P.push_back(pos[q]); }
                else lpos[l * 4 + q] = static_cast<int>(it - P.begin());
              }
            }
            const int sp = static_cast<int>(P.size());
            // Delta on P and its derivative (only link ellk moves)
            std::vector<cplx> Dl(sp * sp, 0.0), dDl(sp * sp, 0.0), Rp(sp * sp, 0.0);
            cplx dov = 0.0, ovk = 1.0, den = 0.0, deq[16], dgk[16];
            int kl = -1;
            for (int l = 0; l < nl; ++l) {
              Even2 ket, bra;
              vectors(links[l], n, m, ket, bra);
              cplx g[16], dg[16], nb, q[16];
              transition_cov(bra, ket, g);
              occupation_response(bra, ket, nb, q);
              const int lv = static_cast<int>(br[14 + (links[l] == d->patch_link[n] && n > 0 ? n : m)]);
              cplx dgl[16], blk[16];
              for (int i = 0; i < 16; ++i) dgl[i] = g[i] - g0c[i];
              rotate4(dgl, lv, group, blk);
              for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) Dl[lpos[l * 4 + i] * sp + lpos[l * 4 + j]] += blk[i * 4 + j];
              // the pair's own electric response on this link replaces the reference one in R
              if (cp->ke != 0.0) {
                cplx dq[16], qr[16];
                for (int i = 0; i < 16; ++i) dq[i] = q[i] - eq0[i];
                rotate4(dq, lv, group, qr);
                int pos[4];
                link_pos(links[l], pos);
                for (int a = 0; a < sp; ++a)
                  for (int b = 0; b < sp; ++b) {
                    cplx v = 0.0;
                    for (int i = 0; i < 4; ++i)
                      for (int j = 0; j < 4; ++j) v += qr[j * 4 + i] * gss(P[a], pos[i]) * gss(P[b], pos[j]);
                    Rp[a * sp + b] -= 0.5 * cp->ke * v;
                  }
              }
              if (links[l] == ellk) {
                kl = l;
                Even2 dket{0.0, 0.0}, dbra{0.0, 0.0};
                if (n == k) dket = db;
                if (m == k) dbra = db;
                cplx dgr[16];
                transition_derivative(bra, ket, dbra, dket, dg, dov, den, deq);
                rotate4(dg, lv, group, dgr);
                for (int i = 0; i < 16; ++i) dgk[i] = dgr[i];
                for (int i = 0; i < 4; ++i)
                  for (int j = 0; j < 4; ++j) dDl[lpos[l * 4 + i] * sp + lpos[l * 4 + j]] += dgr[i * 4 + j];
                ovk = std::conj(bra.a) * ket.a + std::conj(bra.b) * ket.b;
              }
            }
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) Rp[a * sp + b] += R(P[a], P[b]);
            // A = 1 + G_PP Delta, Y = Delta A^-1, M^-1_PP = G_PP - G_PP Y G_PP
            std::vector<cplx> A(sp * sp), Ai;
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) {
                cplx v = (a == b) ? 1.0 : 0.0;
                for (int q = 0; q < sp; ++q) v += gss(P[a], P[q]) * Dl[q * sp + b];
                A[a * sp + b] = v;
              }
            Ai = A;
            if (!cinvert(Ai, sp)) return fail(ctx, GGF_ENONFINITE, "singular pair capacitance in row " + std::to_string(r));
            std::vector<cplx> Y(sp * sp, 0.0), GY(sp * sp, 0.0), Mi(sp * sp, 0.0);
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b)
                for (int q = 0; q < sp; ++q) Y[a * sp + b] += Dl[a * sp + q] * Ai[q * sp + b];
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b)
                for (int q = 0; q < sp; ++q) GY[a * sp + b] += gss(P[a], P[q]) * Y[q * sp + b];
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) {
                cplx v = gss(P[a], P[b]);
                for (int q = 0; q < sp; ++q) v -= GY[a * sp + q] * gss(P[q], P[b]);
                Mi[a * sp + b] = v;
              }
            // d log r = (1/2) tr(M^-1 dM)
            cplx dlogr = 0.0;
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) dlogr += 0.5 * Mi[a * sp + b] * dDl[b * sp + a];
            // dY = (1 - Y G_PP) dDelta A^-1
            std::vector<cplx> T1(sp * sp, 0.0), dY(sp * sp, 0.0);
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) {
                cplx v = 0.0;
                for (int q = 0; q < sp; ++q) v += dDl[a * sp + q] * Ai[q * sp + b];
                T1[a * sp + b] = v;
              }
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) {
                cplx v = T1[a * sp + b];
                for (int q = 0; q < sp; ++q) {
                  cplx yg = 0.0;
                  for (int t = 0; t < sp; ++t) yg += Y[a * sp + t] * gss(P[t], P[q]);
                  v -= yg * T1[q * sp + b];
                }
                dY[a * sp + b] = v;
              }
            cplx dh = 0.0;
            for (int a = 0; a < sp; ++a)
              for (int b = 0; b < sp; ++b) dh -= dY[a * sp + b] * Rp[a * sp + b];
            if (cp->ke != 0.0 && kl >= 0) {
              // explicit change of the varied link's mixed occupation: d en + (1/2) tr(M^-1_UU O deq O^T)
              cplx dqr[16];
              rotate4(deq, kv, group, dqr);
              cplx x = den;
              for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) x += 0.5 * Mi[lpos[kl * 4 + i] * sp + lpos[kl * 4 + j]] * dqr[j * 4 + i];
              dh += cp->ke * x;
            }
            const cplx dlogrho = dov / ovk + dlogr;
            dN += om[p] / Ssum * dlogrho;
            dE += om[p] / Ssum * (dh + (h[p] - e / Ssum) * dlogrho);
          }
        de[r * nout + (k - 1) * ng + gi] = dE.real();
        dn[r * nout + (k - 1) * ng + gi] = dN.real();
      }
    }
  }
  double ebar = 0.0;
  for (int64_t r = 0; r < n_rows; ++r) {
    if (!std::isfinite(es[r])) return fail(ctx, GGF_ENONFINITE, "non-finite energy in row " + std::to_string(r));
    ebar += es[r];
  }
  ebar /= static_cast<double>(n_rows);
  for (int q = 0; q < nout; ++q) {
    double acc = 0.0;
    for (int64_t r = 0; r < n_rows; ++r) acc += de[r * nout + q] + (es[r] - ebar) * dn[r * nout + q];
    grad[q] = acc / static_cast<double>(n_rows);
    if (!std::isfinite(grad[q])) return fail(ctx, GGF_ENONFINITE, "non-finite bond gradient");
  }
  return GGF_OK;
}

namespace {

// Eigenpairs of a real symmetric matrix (order <= 2 GGF_KMAX) by cyclic Jacobi rotations;
// a is destroyed, v receives the eigenvectors as columns, w the eigenvalues.
void jacobi_eigen(int m, double *a, double *v, double *w) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) v[i * m + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += a[i * m + j] * a[i * m + j];
    if (off < 1e-30) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = a[p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {   // columns p, q
          const double akp = a[k * m + p], akq = a[k * m + q];
          a[k * m + p] = c * akp - s * akq;
          a[k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {   // rows p, q
          const double apk = a[p * m + k], aqk = a[q * m + k];
          a[p * m + k] = c * apk - s * aqk;
          a[q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = v[k * m + p], vkq = v[k * m + q];
          v[k * m + p] = c * vkp - s * vkq;
          v[k * m + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < m; ++i) w[i] = a[i * m + i];
}

}  // namespace

ggf_status ggf_lambda_step(ggf_ctx *ctx, int32_t K, const double *rows, int64_t n_rows, double *energy,
                           double *lambda_re, double *lambda_im) {
  if (K < 1 || K > GGF_KMAX) return fail(ctx, GGF_EINVAL, "K must be in 1..GGF_KMAX");
  if (!rows || n_rows <= 0 || !energy || !lambda_re || !lambda_im)
    return fail(ctx, GGF_EINVAL, "rows, n_rows > 0, energy and lambda are required");
  // Hb = mean of rho h / S, Nb = mean of rho / S (Hermitian parts)
  std::vector<cplx> Hb(K * K, 0.0), Nb(K * K, 0.0);
  for (int64_t r = 0; r < n_rows; ++r) {
    const double *row = rows + r * GGF_ENERGY_STRIDE;
    for (int p = 0; p < K * K; ++p) {
      const cplx rho(row[1 + 4 * p], row[2 + 4 * p]), rh(row[3 + 4 * p], row[4 + 4 * p]);
      if (!std::isfinite(rho.real()) || !std::isfinite(rho.imag()) || !std::isfinite(rh.real()) ||
          !std::isfinite(rh.imag()))
        return fail(ctx, GGF_ENONFINITE, "non-finite pair matrices in row " + std::to_string(r));
      Nb[p] += rho;
      Hb[p] += rh;
    }
  }
  std::vector<cplx> H(K * K), S(K * K);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) {
      H[i * K + j] = 0.5 * (Hb[i * K + j] + std::conj(Hb[j * K + i])) / static_cast<double>(n_rows);
      S[i * K + j] = 0.5 * (Nb[i * K + j] + std::conj(Nb[j * K + i])) / static_cast<double>(n_rows);
    }
  // Cholesky S = C C^+ (lower C)
  std::vector<cplx> C(K * K, 0.0);
  for (int j = 0; j < K; ++j) {
    double d = S[j * K + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(C[j * K + k]);
    if (!(d > 0.0)) return fail(ctx, GGF_ESINGULAR, "overlap matrix of the superposition is not positive definite");
    C[j * K + j] = std::sqrt(d);
    for (int i = j + 1; i < K; ++i) {
      cplx v = S[i * K + j];
      for (int k = 0; k < j; ++k) v -= C[i * K + k] * std::conj(C[j * K + k]);
      C[i * K + j] = v / C[j * K + j];
    }
  }
  // Ci = C^-1 (lower triangular), A = Ci H Ci^+
  std::vector<cplx> Ci(K * K, 0.0);
  for (int j = 0; j < K; ++j) {
    Ci[j * K + j] = 1.0 / C[j * K + j];
    for (int i = j + 1; i < K; ++i) {
      cplx v = 0.0;
      for (int k = j; k < i; ++k) v -= C[i * K + k] * Ci[k * K + j];
      Ci[i * K + j] = v / C[i * K + i];
    }
  }
  std::vector<cplx> T(K * K, 0.0), A(K * K, 0.0);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j)
      for (int k = 0; k < K; ++k) T[i * K + j] += Ci[i * K + k] * H[k * K + j];
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j)
      for (int k = 0; k < K; ++k) A[i * K + j] += T[i * K + k] * std::conj(Ci[j * K + k]);
  // Hermitian A as the real symmetric [[Re, -Im], [Im, Re]] (each eigenvalue twice)
  const int m = 2 * K;
  std::vector<double> R(m * m), Vv(m * m), w(m);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) {
      const cplx z = A[i * K + j];
      R[i * m + j] = z.real();
      R[i * m + K + j] = -z.imag();
      R[(K + i) * m + j] = z.imag();
      R[(K + i) * m + K + j] = z.real();
    }
  jacobi_eigen(m, R.data(), Vv.data(), w.data());
  int lo = 0;
  for (int i = 1; i < m; ++i)
    if (w[i] < w[lo]) lo = i;
  std::vector<cplx> y(K), lam(K, 0.0);
  for (int i = 0; i < K; ++i) y[i] = cplx(Vv[i * m + lo], Vv[(K + i) * m + lo]);
  double ny = 0.0;
  for (int i = 0; i < K; ++i) ny += std::norm(y[i]);
  for (int i = 0; i < K; ++i) y[i] /= std::sqrt(ny);
  // lambda = Ci^+ y, so lambda^+ S lambda = 1; phase with lambda_0 real and positive
  for (int i = 0; i < K; ++i)
    for (int k = 0; k < K; ++k) lam[i] += std::conj(Ci[k * K + i]) * y[k];
  const cplx ph = std::abs(lam[0]) > 0 ? std::conj(lam[0]) / std::abs(lam[0]) : cplx(1.0, 0.0);
  for (int i = 0; i < K; ++i) {
    lambda_re[i] = (lam[i] * ph).real();
    lambda_im[i] = (lam[i] * ph).imag();
  }
  *energy = w[lo];
  return GGF_OK;
}

ggf_status ggf_optimise_lambda(ggf_ctx *ctx, int32_t tensor_id, const ggf_couplings *cp, int32_t n_iters,
                               int32_t n_sweeps, double *energies, double *e_opt, double *lambda_re,
                               double *lambda_im, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (tensor_id < 0 || tensor_id >= static_cast<int32_t>(ctx->tensors.size()))
    return fail(ctx, GGF_EINVAL, "bad tensor id");
  if (!cp || n_iters < 1 || n_sweeps < 1 || !energies || !e_opt || !lambda_re || !lambda_im)
    return fail(ctx, GGF_EINVAL, "couplings, n_iters >= 1, n_sweeps >= 1 and the outputs are required");
  const int K = ctx->tensors[tensor_id].K;
  std::vector<int> which;
  for (int c = 0; c < ctx->n_chains; ++c)
    if (ctx->chains[c].tensor == tensor_id) which.push_back(c);
  if (which.empty()) return fail(ctx, GGF_EINVAL, "no chain uses this tensor");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t row_bytes = static_cast<size_t>(ctx->n_chains) * GGF_ENERGY_STRIDE * sizeof(double);
  double *dev = nullptr;
  HIP_TRY(ctx, hipMalloc(&dev, row_bytes * n_sweeps));
  std::vector<double> host(static_cast<size_t>(ctx->n_chains) * GGF_ENERGY_STRIDE * n_sweeps);
  std::vector<double> rows(which.size() * GGF_ENERGY_STRIDE * n_sweeps);
  ggf_status st = GGF_OK;
  for (int it = 0; it < n_iters && st == GGF_OK; ++it) {
    for (int sw = 0; sw < n_sweeps && st == GGF_OK; ++sw) {
      st = ggf_sweep(ctx, 1, stream);
      if (st == GGF_OK)
        st = ggf_measure_energy(ctx, cp, dev + static_cast<size_t>(sw) * ctx->n_chains * GGF_ENERGY_STRIDE, 1,
                                stream);
    }
    if (st != GGF_OK) break;
    hipError_t e = hipMemcpyAsync(host.data(), dev, row_bytes * n_sweeps, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = fail(ctx, GGF_EDEVICE, std::string("optimise_lambda: ") + hipGetErrorString(e));
      break;
    }
    double esum = 0.0;
    size_t r = 0;
    for (int sw = 0; sw < n_sweeps; ++sw)
      for (int c : which) {
        const double *src = host.data() + (static_cast<size_t>(sw) * ctx->n_chains + c) * GGF_ENERGY_STRIDE;
        std::copy(src, src + GGF_ENERGY_STRIDE, rows.data() + r * GGF_ENERGY_STRIDE);
        esum += src[0];
        ++r;
      }
    energies[it] = esum / static_cast<double>(r);
    st = ggf_lambda_step(ctx, K, rows.data(), static_cast<int64_t>(r), &e_opt[it], lambda_re, lambda_im);
    if (st == GGF_OK) st = ggf_set_lambda(ctx, tensor_id, lambda_re, lambda_im, stream);
  }
  hipFree(dev);
  return st;
}

ggf_status ggf_measure_sensitivity(ggf_ctx *ctx, const ggf_couplings *cp, double *out, int32_t out_is_device,
                                   void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (!out || !cp) return fail(ctx, GGF_EINVAL, "out and couplings are required");
  const double cv[5] = {cp->t, cp->mu, cp->m, cp->kb, cp->ke};
  for (double v : cv)
    if (!std::isfinite(v)) return fail(ctx, GGF_EINVAL, "couplings must be finite");
  int max_sites = 0, max_n = 0, max_group = 0;
  bool pairs = false;
  for (const ChainDev &ch : ctx->chains) {
    if (ch.K > 1) pairs = true;
    max_sites = std::max(max_sites, ch.L * ch.L);
    max_n = std::max(max_n, ch.n);
    max_group = std::max(max_group, ch.group);
  }
  for (const ChainDev &ch : ctx->chains)
    if (ch.L > 32) return fail(ctx, GGF_EINVAL, "sensitivities need L <= 32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LaunchCtx lc = launch_ctx(ctx, s);
  const EnergyCp ec{cp->t, cp->mu, cp->m, cp->kb, cp->ke};
  const size_t bytes = static_cast<size_t>(ctx->n_chains) * GGF_SENS_STRIDE * sizeof(double);
  if (!pairs && out_is_device) {
    ggf_launch_sens(lc, ec, out, max_sites, max_group);
    HIP_TRY(ctx, hipGetLastError());
    return GGF_OK;
  }
  // K > 1: the chains' energy rows (pair weights, h_ab and E) and per chain the pair inverse M_ab^-1
  // (complex n x n) or, for n > 512, the factors of its correction to G
  double *tmp = nullptr, *erows = nullptr;
  void *gab = nullptr;
  hipError_t e = out_is_device ? hipSuccess : hipMalloc(&tmp, bytes);
  if (e == hipSuccess && pairs)
    e = hipMalloc(&erows, static_cast<size_t>(ctx->n_chains) * GGF_ENERGY_STRIDE * sizeof(double));
  if (e == hipSuccess && pairs)
    e = hipMalloc(&gab, ggf_sens_pairs_scratch(ctx->n_chains, max_n));
  double *dst = out_is_device ? out : tmp;
  if (e == hipSuccess) {
    if (pairs) {
      ggf_launch_energy(lc, ec, erows, ctx->kmax);
      ggf_launch_sens_pairs(lc, ec, gab, max_n, erows, dst, ctx->kmax);
    } else {
      ggf_launch_sens(lc, ec, dst, max_sites, max_group);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess && !out_is_device) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && (pairs || !out_is_device)) e = hipStreamSynchronize(s);
  if (tmp) hipFree(tmp);
  if (erows) hipFree(erows);
  if (gab) hipFree(gab);
  if (e != hipSuccess) return fail(ctx, GGF_EDEVICE, std::string("measure_sensitivity: ") + hipGetErrorString(e));
  return GGF_OK;
}

ggf_status ggf_gamma_gradient(ggf_ctx *ctx, const double *gamma_loc, const double *energy_rows,
                              const double *sens_rows, int64_t n_rows, double *grad) {
  if (!gamma_loc || !energy_rows || !sens_rows || n_rows <= 0 || !grad)
    return fail(ctx, GGF_EINVAL, "gamma_loc, rows, n_rows > 0 and grad are required");
  double ebar = 0.0;
  for (int64_t r = 0; r < n_rows; ++r) {
    const double e = energy_rows[r * GGF_ENERGY_STRIDE];
    if (!std::isfinite(e)) return fail(ctx, GGF_ENONFINITE, "non-finite energy in row " + std::to_string(r));
    ebar += e;
  }
  ebar /= static_cast<double>(n_rows);
  // Sbar = mean S_e + mean (e - ebar) S_N
  double S[100] = {0.0};
  for (int64_t r = 0; r < n_rows; ++r) {
    const double de = energy_rows[r * GGF_ENERGY_STRIDE] - ebar;
    const double *row = sens_rows + r * GGF_SENS_STRIDE;
    for (int q = 0; q < 100; ++q) {
      if (!std::isfinite(row[q]) || !std::isfinite(row[100 + q]))
        return fail(ctx, GGF_ENONFINITE, "non-finite sensitivity in row " + std::to_string(r));
      S[q] += row[q] + de * row[100 + q];
    }
  }
  for (double &v : S) v /= static_cast<double>(n_rows);
  // d<H>/d theta_kl = tr([E_kl, Gamma] S) = Y[l][k] - Y[k][l], Y = Gamma S - S Gamma
  double Y[100];
  for (int i = 0; i < 10; ++i)
    for (int j = 0; j < 10; ++j) {
      double v = 0.0;
      for (int k = 0; k < 10; ++k) v += gamma_loc[i * 10 + k] * S[k * 10 + j] - S[i * 10 + k] * gamma_loc[k * 10 + j];
      Y[i * 10 + j] = v;
    }
  for (int k = 0; k < 10; ++k)
    for (int l = 0; l < 10; ++l) grad[k * 10 + l] = Y[l * 10 + k] - Y[k * 10 + l];
  return GGF_OK;
}

ggf_status ggf_set_gamma_loc(ggf_ctx *ctx, int32_t tensor_id, const double *gamma_loc, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (tensor_id < 0 || tensor_id >= static_cast<int32_t>(ctx->tensors.size()))
    return fail(ctx, GGF_EINVAL, "bad tensor id");
  if (!gamma_loc) return fail(ctx, GGF_EINVAL, "gamma_loc is required");
  std::string why;
  if (!check_local(gamma_loc, why)) return fail(ctx, GGF_EINVAL, why);
  TensorDev &t = ctx->tensors[tensor_id];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) t.a[i * 2 + j] = gamma_loc[i * 10 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 8; ++j) t.b[i * 8 + j] = gamma_loc[i * 10 + 2 + j];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) t.d[i * 8 + j] = gamma_loc[(2 + i) * 10 + 2 + j];
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->tensors_dev + tensor_id, &t, sizeof(TensorDev), hipMemcpyHostToDevice, s));
  std::vector<int> which;
  for (int c = 0; c < ctx->n_chains; ++c)
    if (ctx->chains[c].tensor == tensor_id) which.push_back(c);
  if (which.empty()) {
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return GGF_OK;
  }
  return factorize(ctx, which, 0, s);
}

namespace {

// exp(X) of a real 10 x 10 matrix by scaling and squaring with a degree-16 Taylor polynomial
// (X antisymmetric here, so the result is a rotation to rounding).
void expm10(const double *X, double *R) {
  double nrm = 0.0;
  for (int i = 0; i < 100; ++i) nrm = std::max(nrm, std::fabs(X[i]));
  int sq = 0;
  while (nrm * 10.0 > 0.25 && sq < 60) { nrm *= 0.5; ++sq; }
  const double scale = std::ldexp(1.0, -sq);
  double A[100], T[100], U[100];
  for (int i = 0; i < 100; ++i) { A[i] = X[i] * scale; R[i] = (i % 11 == 0) ? 1.0 : 0.0; T[i] = R[i]; }
  for (int k = 1; k <= 16; ++k) {
    for (int i = 0; i < 10; ++i)
      for (int j = 0; j < 10; ++j) {
        double v = 0.0;
        for (int q = 0; q < 10; ++q) v += T[i * 10 + q] * A[q * 10 + j];
        U[i * 10 + j] = v / k;
      }
    for (int i = 0; i < 100; ++i) { T[i] = U[i]; R[i] += U[i]; }
  }
  for (int s2 = 0; s2 < sq; ++s2) {
    for (int i = 0; i < 10; ++i)
      for (int j = 0; j < 10; ++j) {
        double v = 0.0;
        for (int q = 0; q < 10; ++q) v += R[i * 10 + q] * R[q * 10 + j];
        U[i * 10 + j] = v;
      }
    for (int i = 0; i < 100; ++i) R[i] = U[i];
  }
}

}  // namespace

ggf_status ggf_optimise_gamma(ggf_ctx *ctx, int32_t tensor_id, const ggf_couplings *cp, int32_t n_iters,
                              int32_t n_sweeps, double step, double *energies, double *grad_norms,
                              double *gamma_loc_out, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (tensor_id < 0 || tensor_id >= static_cast<int32_t>(ctx->tensors.size()))
    return fail(ctx, GGF_EINVAL, "bad tensor id");
  if (!cp || n_iters < 1 || n_sweeps < 1 || !(std::isfinite(step) && step > 0.0) || !energies || !grad_norms ||
      !gamma_loc_out)
    return fail(ctx, GGF_EINVAL, "couplings, n_iters >= 1, n_sweeps >= 1, step > 0 and the outputs are required");
  std::vector<int> which;
  for (int c = 0; c < ctx->n_chains; ++c)
    if (ctx->chains[c].tensor == tensor_id) which.push_back(c);
  if (which.empty()) return fail(ctx, GGF_EINVAL, "no chain uses this tensor");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nc = static_cast<size_t>(ctx->n_chains);
  double *dev_e = nullptr, *dev_s = nullptr;
  HIP_TRY(ctx, hipMalloc(&dev_e, nc * GGF_ENERGY_STRIDE * sizeof(double) * n_sweeps));
  hipError_t ea = hipMalloc(&dev_s, nc * GGF_SENS_STRIDE * sizeof(double) * n_sweeps);
  if (ea != hipSuccess) {
    hipFree(dev_e);
    return fail(ctx, GGF_EDEVICE, std::string("optimise_gamma: ") + hipGetErrorString(ea));
  }
  std::vector<double> he(nc * GGF_ENERGY_STRIDE * n_sweeps), hs(nc * GGF_SENS_STRIDE * n_sweeps);
  std::vector<double> re(which.size() * GGF_ENERGY_STRIDE * n_sweeps), rs(which.size() * GGF_SENS_STRIDE * n_sweeps);
  ggf_status st = GGF_OK;
  for (int it = 0; it < n_iters && st == GGF_OK; ++it) {
    for (int sw = 0; sw < n_sweeps && st == GGF_OK; ++sw) {
      st = ggf_sweep(ctx, 1, stream);
      if (st == GGF_OK) st = ggf_measure_energy(ctx, cp, dev_e + sw * nc * GGF_ENERGY_STRIDE, 1, stream);
      if (st == GGF_OK) st = ggf_measure_sensitivity(ctx, cp, dev_s + sw * nc * GGF_SENS_STRIDE, 1, stream);
    }
    if (st != GGF_OK) break;
    hipError_t e = hipMemcpyAsync(he.data(), dev_e, he.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), dev_s, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = fail(ctx, GGF_EDEVICE, std::string("optimise_gamma: ") + hipGetErrorString(e));
      break;
    }
    size_t r = 0;
    double esum = 0.0;
    for (int sw = 0; sw < n_sweeps; ++sw)
      for (int c : which) {
        const double *se = he.data() + (sw * nc + c) * GGF_ENERGY_STRIDE;
        const double *ss = hs.data() + (sw * nc + c) * GGF_SENS_STRIDE;
        std::copy(se, se + GGF_ENERGY_STRIDE, re.data() + r * GGF_ENERGY_STRIDE);
        std::copy(ss, ss + GGF_SENS_STRIDE, rs.data() + r * GGF_SENS_STRIDE);
        esum += se[0];
        ++r;
      }
    energies[it] = esum / static_cast<double>(r);
    // current Gamma_A of the tensor
    const TensorDev &t = ctx->tensors[tensor_id];
    double gam[100], grad[100], X[100], R[100], nxt[100];
    for (int i = 0; i < 100; ++i) gam[i] = 0.0;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) gam[i * 10 + j] = t.a[i * 2 + j];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 8; ++j) {
        gam[i * 10 + 2 + j] = t.b[i * 8 + j];
        gam[(2 + j) * 10 + i] = -t.b[i * 8 + j];
      }
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) gam[(2 + i) * 10 + 2 + j] = t.d[i * 8 + j];
    st = ggf_gamma_gradient(ctx, gam, re.data(), rs.data(), static_cast<int64_t>(r), grad);
    if (st != GGF_OK) break;
    double gn = 0.0;
    for (int i = 0; i < 100; ++i) gn = std::max(gn, std::fabs(grad[i]));
    grad_norms[it] = gn;
    // descent step: theta_kl = -step g_kl, Gamma <- exp(X) Gamma exp(-X), X = -step g
    for (int i = 0; i < 100; ++i) X[i] = -step * grad[i];
    expm10(X, R);
    for (int i = 0; i < 10; ++i)
      for (int j = 0; j < 10; ++j) {
        double v = 0.0;
        for (int p = 0; p < 10; ++p)
          for (int q = 0; q < 10; ++q) v += R[i * 10 + p] * gam[p * 10 + q] * R[j * 10 + q];
        nxt[i * 10 + j] = v;
      }
    for (int i = 0; i < 10; ++i)   // exact antisymmetry (the purity check allows 1e-8)
      for (int j = 0; j < 10; ++j) gamma_loc_out[i * 10 + j] = 0.5 * (nxt[i * 10 + j] - nxt[j * 10 + i]);
    st = ggf_set_gamma_loc(ctx, tensor_id, gamma_loc_out, stream);
  }
  hipFree(dev_e);
  hipFree(dev_s);
  return st;
}

ggf_status ggf_get_state(ggf_ctx *ctx, int32_t chain, int8_t *links, ggf_chain_info *info) {
  if (!ctx) return GGF_EINVAL;
  if (chain < 0 || chain >= ctx->n_chains) return fail(ctx, GGF_EINVAL, "chain index out of range");
  HIP_TRY(ctx, hipDeviceSynchronize());
  const ChainDev &d = ctx->chains[chain];
  if (links) HIP_TRY(ctx, hipMemcpy(links, ctx->links + d.link_off, d.nlinks, hipMemcpyDeviceToHost));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->L = d.L;
    info->n = d.n;
    info->tensor_id = d.tensor;
    info->precision = ctx->precision;
    double2 sf;
    uint32_t sw;
    HIP_TRY(ctx, hipMemcpy(&info->logw, ctx->logw + chain, sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&sf, ctx->sfac + chain, sizeof(double2), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&sw, ctx->sweep + chain, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&info->accepts, ctx->acc_total + chain, sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&info->proposals, ctx->prop_total + chain, sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&info->refreshes, ctx->refreshes + chain, sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&info->max_drift, ctx->max_drift + chain, sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&info->near_ties, ctx->ties + chain, sizeof(uint64_t), hipMemcpyDeviceToHost));
    int cur = 0;
    HIP_TRY(ctx, hipMemcpy(&cur, ctx->cursor + chain, sizeof(int), hipMemcpyDeviceToHost));
    info->link_cursor = static_cast<uint64_t>(cur);
    info->s_re = sf.x;
    info->s_im = sf.y;
    info->sweeps = sw;
    info->recoveries = ctx->recoveries[chain];
  }
  return GGF_OK;
}

ggf_status ggf_set_state(ggf_ctx *ctx, int32_t chain, const int8_t *links, uint64_t sweeps) {
  if (!ctx) return GGF_EINVAL;
  if (chain < 0 || chain >= ctx->n_chains) return fail(ctx, GGF_EINVAL, "chain index out of range");
  if (!links) return fail(ctx, GGF_EINVAL, "links is NULL");
  if (sweeps > 0xFFFFFFFEull) return fail(ctx, GGF_EINVAL, "sweep counter out of range");
  const ChainDev &d = ctx->chains[chain];
  for (int l = 0; l < d.nlinks; ++l)
    if (links[l] < 0 || links[l] >= d.group) return fail(ctx, GGF_EINVAL, "link value outside Z_N");
  HIP_TRY(ctx, hipDeviceSynchronize());
  HIP_TRY(ctx, hipMemcpy(ctx->links + d.link_off, links, d.nlinks, hipMemcpyHostToDevice));
  const uint32_t sw = static_cast<uint32_t>(sweeps);
  HIP_TRY(ctx, hipMemcpy(ctx->sweep + chain, &sw, sizeof(uint32_t), hipMemcpyHostToDevice));
  const int zero = 0;
  HIP_TRY(ctx, hipMemcpy(ctx->flags + chain, &zero, sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->cursor + chain, &zero, sizeof(int), hipMemcpyHostToDevice));   // a sweep boundary
  return factorize(ctx, std::vector<int>{chain}, 0, nullptr);
}

ggf_status ggf_get_inverse(ggf_ctx *ctx, int32_t chain, double *host_out) {
  if (!ctx) return GGF_EINVAL;
  if (chain < 0 || chain >= ctx->n_chains) return fail(ctx, GGF_EINVAL, "chain index out of range");
  if (!host_out) return fail(ctx, GGF_EINVAL, "host_out is NULL");
  HIP_TRY(ctx, hipDeviceSynchronize());
  const ChainDev &d = ctx->chains[chain];
  const size_t nn = static_cast<size_t>(d.n) * d.n;
  if (ctx->precision == 64) {
    HIP_TRY(ctx, hipMemcpy(host_out, static_cast<double *>(ctx->G) + d.g_off, nn * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(nn);
    HIP_TRY(ctx, hipMemcpy(tmp.data(), static_cast<float *>(ctx->G) + d.g_off, nn * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < nn; ++i) host_out[i] = tmp[i];
  }
  return GGF_OK;
}

ggf_status ggf_set_inverse(ggf_ctx *ctx, int32_t chain, const double *host_in) {
  if (!ctx) return GGF_EINVAL;
  if (chain < 0 || chain >= ctx->n_chains) return fail(ctx, GGF_EINVAL, "chain index out of range");
  if (!host_in) return fail(ctx, GGF_EINVAL, "host_in is NULL");
  HIP_TRY(ctx, hipDeviceSynchronize());
  const ChainDev &d = ctx->chains[chain];
  const size_t nn = static_cast<size_t>(d.n) * d.n;
  if (ctx->precision == 64) {
    HIP_TRY(ctx, hipMemcpy(static_cast<double *>(ctx->G) + d.g_off, host_in, nn * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::vector<float> tmp(host_in, host_in + nn);
    HIP_TRY(ctx, hipMemcpy(static_cast<float *>(ctx->G) + d.g_off, tmp.data(), nn * sizeof(float), hipMemcpyHostToDevice));
  }
  return GGF_OK;
}

ggf_status ggf_refresh_all(ggf_ctx *ctx, void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  std::vector<int> all(ctx->n_chains);
  for (int c = 0; c < ctx->n_chains; ++c) all[c] = c;
  return factorize(ctx, all, 1, static_cast<hipStream_t>(stream));
}

ggf_status ggf_set_option(ggf_ctx *ctx, const char *key, int64_t value) {
  if (!ctx || !key) return GGF_EINVAL;
  const std::string k(key);
  if (value < 0) return fail(ctx, GGF_EINVAL, "option values must be >= 0");
  if (k == "update_grid") ctx->opt_update_grid = static_cast<int>(value);
  else if (k == "update_tiles") ctx->opt_update_tiles = static_cast<int>(value);
  else if (k == "graph") {
    ctx->opt_graph = value != 0;
    if (ctx->graph_exec) { hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
  } else if (k == "gj_nb") {
    if (value != 0 && (value < 8 || value > 256)) return fail(ctx, GGF_EINVAL, "gj_nb must be in 8..256");
    ctx->opt_gj_nb = static_cast<int>(value);
  } else if (k == "scratch_mb") ctx->opt_scratch_mb = value;
  else if (k == "time_update") ctx->opt_time_update = value != 0;
  else if (k == "update_nt") ctx->opt_update_nt = value != 0;
  else if (k == "flush_grid") ctx->opt_flush_grid = static_cast<int>(std::min<int64_t>(value, 1 << 20));
  else if (k == "block_pend") {
    if (value > GGF_BLOCK_RMAX) return fail(ctx, GGF_EINVAL, "block_pend must be in 0..128");
    ctx->opt_block_pend = static_cast<int>(value);
  } else if (k == "block_rho") {
    if (value < 1 || value > 65536) return fail(ctx, GGF_EINVAL, "block_rho must be in 1..65536 (units of 1/65536)");
    ctx->opt_block_rho = static_cast<int>(value);
  }
  else if (k == "balance") {
    if (value > 1) return fail(ctx, GGF_EINVAL, "balance must be 0 or 1");
    if (ctx->n_chains > 0 && !ctx->opt_balance && value) {
      // chains enter balanced sweeps at the start of a sweep
      HIP_TRY(ctx, hipMemset(ctx->cursor, 0, ctx->n_chains * sizeof(int)));
    }
    if (ctx->n_chains > 0 && ctx->opt_balance && !value) {
      std::vector<int> cur(ctx->n_chains);
      HIP_TRY(ctx, hipMemcpy(cur.data(), ctx->cursor, cur.size() * sizeof(int), hipMemcpyDeviceToHost));
      for (int v : cur)
        if (v != 0) return fail(ctx, GGF_ESTATE, "balanced sweeps can end only when every chain is at a sweep boundary");
    }
    ctx->opt_balance = static_cast<int>(value);
  }
  else if (k == "delay") {
    if (!(value == -1 || value == 0 || (value % 8 == 0 && value >= 8 && value <= 32)))
      return fail(ctx, GGF_EINVAL, "delay must be -1 (automatic), 0 (immediate) or 8, 16, 24, 32 link steps");
    ctx->opt_delay = static_cast<int>(value);
  } else return fail(ctx, GGF_EINVAL, "unknown option " + k);
  if (k == "update_grid" || k == "update_tiles" || k == "update_nt" || k == "delay" || k == "flush_grid" ||
      k == "balance") {
    if (ctx->graph_exec) { hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
  }
  return GGF_OK;
}

ggf_status ggf_autotune(ggf_ctx *ctx, int32_t sweeps_per_candidate, const char *cache_path, int64_t *best,
                        void *stream) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->n_chains == 0) return fail(ctx, GGF_ESTATE, "ggf_init_chains has not been called");
  if (sweeps_per_candidate < 1) return fail(ctx, GGF_EINVAL, "sweeps_per_candidate must be >= 1");
  // delayed updates (the default): the flush grid and the window length; immediate updates
  // (delay = 0): the launch shape of the rank-4 streaming update
  const bool delayed = delay_window(ctx) > 0;
  char key[160];
  std::snprintf(key, sizeof(key), "%s_n%d_p%d_K%d_c%d", delayed ? "flush" : "update", ctx->n_max, ctx->precision,
                ctx->kmax, ctx->n_chains);
  long long choice[3] = {0, 0, 0};
  bool found = false;
  if (cache_path) {
    if (FILE *f = std::fopen(cache_path, "r")) {
      char k[160];
      long long a, b, c;
      while (std::fscanf(f, "%159s %lld %lld %lld", k, &a, &b, &c) == 4)
        if (std::strcmp(k, key) == 0) { choice[0] = a; choice[1] = b; choice[2] = c; found = true; }
      std::fclose(f);
    }
  }
  if (!found) {
    const int saved_time = ctx->opt_time_update;
    ctx->opt_time_update = 1;
    double best_cost = 1e300;
    auto timed_cost = [&](double &cost) -> ggf_status {
      ggf_status st = ggf_sweep(ctx, sweeps_per_candidate, stream);
      if (st != GGF_OK) return st;
      const double props = static_cast<double>(sweeps_per_candidate) * ctx->max_links * ctx->n_chains;
      // link steps and update launches: the part of a sweep the launch shape changes
      cost = (ctx->last_update_ms + ctx->last_ratio_ms) / props;
      return GGF_OK;
    };
    if (delayed) {
      const int grids[3] = {512, 1024, 2048};
      const int windows[3] = {8, 16, 32};
      for (int wi = 0; wi < 3; ++wi)
        for (int gi = 0; gi < 3; ++gi) {
          ctx->opt_delay = windows[wi];
          ctx->opt_flush_grid = grids[gi];
          double cost = 0.0;
          ggf_status st = timed_cost(cost);
          if (st != GGF_OK) return st;
          if (cost < best_cost) {
            best_cost = cost;
            choice[0] = grids[gi];
            choice[1] = windows[wi];
            choice[2] = 0;
          }
        }
    } else {
      const int grids[3] = {1024, 2048, 4096};
      const int rows[3] = {8, 16, 32};
      for (int nt = 1; nt >= 0; --nt)
        for (int gi = 0; gi < 3; ++gi)
          for (int ri = 0; ri < 3; ++ri) {
            ctx->opt_update_grid = grids[gi];
            ctx->opt_update_tiles = std::max(1, ctx->n_max / rows[ri]);
            ctx->opt_update_nt = nt;
            double cost = 0.0;
            ggf_status st = timed_cost(cost);
            if (st != GGF_OK) return st;
            if (cost < best_cost) {
              best_cost = cost;
              choice[0] = grids[gi];
              choice[1] = ctx->opt_update_tiles;
              choice[2] = nt;
            }
          }
    }
    ctx->opt_time_update = saved_time;
    if (cache_path && choice[0] > 0) {
      if (FILE *f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %lld %lld %lld\n", key, choice[0], choice[1], choice[2]);
        std::fclose(f);
      }
    }
  }
  if (choice[0] > 0) {
    if (delayed) {
      ctx->opt_flush_grid = static_cast<int>(choice[0]);
      ctx->opt_delay = static_cast<int>(choice[1]);
    } else {
      ctx->opt_update_grid = static_cast<int>(choice[0]);
      ctx->opt_update_tiles = static_cast<int>(choice[1]);
      ctx->opt_update_nt = static_cast<int>(choice[2]);
    }
    if (ctx->graph_exec) { hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
  }
  if (best)
    for (int q = 0; q < 3; ++q) best[q] = choice[q];
  return GGF_OK;
}

ggf_status ggf_update_timing(ggf_ctx *ctx, double *ms, int64_t *launches, int64_t *flips) {
  if (!ctx) return GGF_EINVAL;
  if (ms) *ms = ctx->last_update_ms;
  if (launches) *launches = ctx->last_launches;
  if (flips) *flips = ctx->last_flips;
  return GGF_OK;
}

ggf_status ggf_ratio_timing(ggf_ctx *ctx, double *ms, int64_t *launches) {
  if (!ctx) return GGF_EINVAL;
  if (ms) *ms = ctx->last_ratio_ms;
  if (launches) *launches = ctx->last_ratio_launches;
  return GGF_OK;
}

ggf_status ggf_autocorr_time(const double *series, int64_t n_t, int64_t n_series, double c, double *tau,
                             double *tau_err, int64_t *window, int32_t *flags) {
  if (!series || n_t < 2 || n_series < 1 || !(c > 0) || !tau) return GGF_EINVAL;
  std::vector<double> x(static_cast<size_t>(n_t) * n_series);
  for (int64_t s = 0; s < n_series; ++s) {
    double m = 0.0;
    for (int64_t t = 0; t < n_t; ++t) m += series[t * n_series + s];
    m /= static_cast<double>(n_t);
    for (int64_t t = 0; t < n_t; ++t) x[t * n_series + s] = series[t * n_series + s] - m;
  }
  std::vector<double> g(n_t, 0.0);
  for (int64_t lag = 0; lag < n_t; ++lag) {
    double acc = 0.0;
    for (int64_t t = 0; t + lag < n_t; ++t)
      for (int64_t s = 0; s < n_series; ++s) acc += x[t * n_series + s] * x[(t + lag) * n_series + s];
    g[lag] = acc / (static_cast<double>(n_t) * n_series);
  }
  double tv = 0.5, err = 0.0;
  int64_t w = 0;
  int32_t fl = 0;
  bool windowed = false;
  if (g[0] > 0) {
    for (int64_t t = 1; t < n_t; ++t) {
      tv += g[t] / g[0];
      w = t;
      if (t >= c * tv) { windowed = true; break; }
    }
    if (tv <= 0.5) fl |= GGF_TAU_FLOOR;
    tv = std::max(tv, 0.5);
    err = tv * std::sqrt(2.0 * (2.0 * w + 1.0) / (static_cast<double>(n_t) * n_series));
  } else {
    fl |= GGF_TAU_FLOOR;
  }
  // centring on each series' own mean biases the autocovariances low by O(tau / n_t): the estimate
  // is only trusted when the series is long against tau and the window
  if (!windowed || static_cast<double>(n_t) < 50.0 * tv || 4 * w > n_t) fl |= GGF_TAU_SHORT;
  *tau = tv;
  if (tau_err) *tau_err = err;
  if (window) *window = w;
  if (flags) *flags = fl;
  return GGF_OK;
}

int32_t ggf_nn_nparams(void) { return GGF_NN_NPARAMS; }

ggf_status ggf_nn_init(ggf_ctx *ctx, int32_t patch, uint64_t seed) {
  if (!ctx) return GGF_EINVAL;
  if (patch != 1 && patch != 2 && patch != 4) return fail(ctx, GGF_EINVAL, "patch side must be 1, 2 or 4");
  if (!ctx->nn_p) {
    hipError_t e = hipSuccess;
    auto grab = [&](size_t bytes) -> void * {
      void *p = nullptr;
      if (e == hipSuccess) e = hipMalloc(&p, std::max<size_t>(bytes, 16));
      if (e == hipSuccess) { ctx->nn_allocs.push_back(p); e = hipMemset(p, 0, std::max<size_t>(bytes, 16)); }
      return p;
    };
    ctx->nn_cap = 65536;
    ctx->nn_p = static_cast<float *>(grab(GGF_NN_NPARAMS * sizeof(float)));
    ctx->nn_m = static_cast<float *>(grab(GGF_NN_NPARAMS * sizeof(float)));
    ctx->nn_v = static_cast<float *>(grab(GGF_NN_NPARAMS * sizeof(float)));
    ctx->nn_g = static_cast<float *>(grab(GGF_NN_NPARAMS * sizeof(float)));
    ctx->nn_gpart = static_cast<float *>(grab(static_cast<size_t>(ctx->nn_nslices) * GGF_NN_NPARAMS * sizeof(float)));
    ctx->nn_wq = static_cast<uint16_t *>(grab(GGF_NN_NPARAMS * sizeof(uint16_t)));
    ctx->nn_lpart = static_cast<double *>(grab(ctx->nn_nslices * sizeof(double)));
    ctx->nn_loss = static_cast<double *>(grab(sizeof(double)));
    ctx->nn_ex_chain = static_cast<int *>(grab(ctx->nn_cap * sizeof(int)));
    ctx->nn_ex_patch = static_cast<int *>(grab(ctx->nn_cap * sizeof(int)));
    ctx->nn_logits = static_cast<float *>(grab(static_cast<size_t>(ctx->nn_cap) * 32 * sizeof(float)));
    if (e != hipSuccess) return fail(ctx, GGF_ENOMEM, "cannot allocate network buffers");
  }
  // Glorot-uniform weights from Philox at counter (index, 0, 0, 9), zero biases
  std::vector<float> p(GGF_NN_NPARAMS, 0.0f);
  const int layers[4][2] = {{2, 32}, {32, 32}, {32, 32}, {32, 2}};
  int off = 0;
  for (int l = 0; l < 4; ++l) {
    const int ci = layers[l][0], co = layers[l][1], cnt = co * ci * 9;
    const double a = std::sqrt(6.0 / (9.0 * ci + 9.0 * co));
    for (int i = 0; i < cnt; ++i) {
      const uint4 x = ggf_philox(make_uint4(static_cast<uint32_t>(off + i), 0u, 0u, 9u),
                                 static_cast<uint32_t>(seed & 0xFFFFFFFFu), static_cast<uint32_t>(seed >> 32));
      const double u = (static_cast<double>(x.x) + 0.5) * 0x1.0p-32;
      p[off + i] = static_cast<float>((2.0 * u - 1.0) * a);
    }
    off += cnt + co;
  }
  ctx->nn_P = patch;
  ctx->nn_adam_t = 0;
  ctx->nn_step = 0;
  HIP_TRY(ctx, hipMemcpy(ctx->nn_p, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemset(ctx->nn_m, 0, GGF_NN_NPARAMS * sizeof(float)));
  HIP_TRY(ctx, hipMemset(ctx->nn_v, 0, GGF_NN_NPARAMS * sizeof(float)));
  ggf_nn_quantize_launch(ctx->nn_p, ctx->nn_wq, nullptr);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipDeviceSynchronize());
  return GGF_OK;
}

ggf_status ggf_nn_params(ggf_ctx *ctx, float *get_host, const float *set_host) {
  if (!ctx) return GGF_EINVAL;
  if (ctx->nn_P == 0) return fail(ctx, GGF_ESTATE, "ggf_nn_init has not been called");
  HIP_TRY(ctx, hipDeviceSynchronize());
  if (get_host) HIP_TRY(ctx, hipMemcpy(get_host, ctx->nn_p, GGF_NN_NPARAMS * sizeof(float), hipMemcpyDeviceToHost));
  if (set_host) {
    HIP_TRY(ctx, hipMemcpy(ctx->nn_p, set_host, GGF_NN_NPARAMS * sizeof(float), hipMemcpyHostToDevice));
    ggf_nn_quantize_launch(ctx->nn_p, ctx->nn_wq, nullptr);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipDeviceSynchronize());
  }
  return GGF_OK;
}

ggf_status ggf_nn_forward(ggf_ctx *ctx, int32_t n, const int32_t *chain, const int32_t *patch, float *logits_host) {
  if (!ctx) return GGF_EINVAL;
  ggf_status st = nn_check_chains(ctx);
  if (st != GGF_OK) return st;
  if (!logits_host) return fail(ctx, GGF_EINVAL, "logits_host is NULL");
  HIP_TRY(ctx, hipDeviceSynchronize());
  if ((st = nn_examples(ctx, n, chain, patch)) != GGF_OK) return st;
  ggf_nn_forward_launch(nn_args(ctx), ctx->nn_ex_chain, ctx->nn_ex_patch, n, ctx->nn_logits, nullptr);
  HIP_TRY(ctx, hipGetLastError());
  const size_t np = 2 * ctx->nn_P * ctx->nn_P;
  HIP_TRY(ctx, hipMemcpy(logits_host, ctx->nn_logits, n * np * sizeof(float), hipMemcpyDeviceToHost));
  return GGF_OK;
}

ggf_status ggf_nn_grad(ggf_ctx *ctx, int32_t n, const int32_t *chain, const int32_t *patch, float *grad_host,
                       double *loss_host) {
  if (!ctx) return GGF_EINVAL;
  ggf_status st = nn_check_chains(ctx);
  if (st != GGF_OK) return st;
  HIP_TRY(ctx, hipDeviceSynchronize());
  if ((st = nn_examples(ctx, n, chain, patch)) != GGF_OK) return st;
  ggf_nn_grad_launch(nn_args(ctx), ctx->nn_ex_chain, ctx->nn_ex_patch, n, ctx->nn_gpart, ctx->nn_nslices,
                     ctx->nn_lpart, ctx->nn_g, ctx->nn_loss, nullptr);
  HIP_TRY(ctx, hipGetLastError());
  if (grad_host) HIP_TRY(ctx, hipMemcpy(grad_host, ctx->nn_g, GGF_NN_NPARAMS * sizeof(float), hipMemcpyDeviceToHost));
  if (loss_host) HIP_TRY(ctx, hipMemcpy(loss_host, ctx->nn_loss, sizeof(double), hipMemcpyDeviceToHost));
  return GGF_OK;
}

ggf_status ggf_nn_train(ggf_ctx *ctx, int32_t steps, int32_t batch, float lr, uint64_t seed, double *loss_host,
                        void *stream) {
  if (!ctx) return GGF_EINVAL;
  ggf_status st = nn_check_chains(ctx);
  if (st != GGF_OK) return st;
  if (steps < 0 || batch <= 0 || batch > ctx->nn_cap || !(lr > 0)) return fail(ctx, GGF_EINVAL, "bad training arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int npatch = 1 << 30;
  for (const ChainDev &c : ctx->chains) npatch = std::min(npatch, (c.L / ctx->nn_P) * (c.L / ctx->nn_P));
  for (int t = 0; t < steps; ++t) {
    ggf_nn_examples_launch(ctx->nn_ex_chain, ctx->nn_ex_patch, batch, ctx->nn_step++,
                           static_cast<uint32_t>(seed & 0xFFFFFFFFu), static_cast<uint32_t>(seed >> 32),
                           ctx->n_chains, npatch, s);
    ggf_nn_grad_launch(nn_args(ctx), ctx->nn_ex_chain, ctx->nn_ex_patch, batch, ctx->nn_gpart, ctx->nn_nslices,
                       ctx->nn_lpart, ctx->nn_g, ctx->nn_loss, s);
    ggf_nn_adam_launch(ctx->nn_p, ctx->nn_wq, ctx->nn_m, ctx->nn_v, ctx->nn_g, lr, ++ctx->nn_adam_t, s);
  }
  HIP_TRY(ctx, hipGetLastError());
  if (loss_host) {
    HIP_TRY(ctx, hipMemcpyAsync(loss_host, ctx->nn_loss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  return GGF_OK;
}

ggf_status ggf_block_sweep(ggf_ctx *ctx, int32_t n_sweeps, void *stream) {
  if (!ctx) return GGF_EINVAL;
  ggf_status st = nn_check_chains(ctx);
  if (st != GGF_OK) return st;
  if (n_sweeps < 0) return fail(ctx, GGF_EINVAL, "n_sweeps must be >= 0");
  if ((st = block_buffers(ctx)) != GGF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int max_np = 0;
  for (const ChainDev &c : ctx->chains) max_np = std::max(max_np, (c.L / ctx->nn_P) * (c.L / ctx->nn_P));
  if (ctx->opt_balance) {
    // block sweeps advance every chain's sweep counter: with balanced single-link sweeps they start
    // only where every chain is at a sweep boundary
    std::vector<int> cur(ctx->n_chains);
    HIP_TRY(ctx, hipMemcpy(cur.data(), ctx->cursor, cur.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (int v : cur)
      if (v != 0) return fail(ctx, GGF_ESTATE, "block sweep while a chain is inside a balanced sweep");
  }
  BlockLaunch bl;
  bl.lc = launch_ctx(ctx, s);
  bl.lc.cursor = nullptr;
  bl.nn = nn_args(ctx);
  bl.A = ctx->blk_A;
  bl.Wf = ctx->blk_W;
  bl.D = ctx->blk_D;
  bl.d_off = ctx->blk_doff;
  bl.U = ctx->blk_U;
  bl.rcnt = ctx->blk_r;
  bl.bprop = ctx->blk_prop;
  bl.bacc = ctx->blk_acc;
  bl.kmax = ctx->kmax;
  bl.pend = ctx->opt_block_pend;
  bl.E = ctx->blk_E;
  bl.Fm = ctx->blk_F;
  bl.Wn = ctx->blk_Wn;
  bl.Un = ctx->blk_Un;
  bl.rn = ctx->blk_rn;
  bl.mode = ctx->blk_mode;
  bl.rho = ctx->opt_block_rho / 65536.0;
  const bool pend = bl.pend > 0;
  const int grid = ctx->opt_update_grid > 0 ? ctx->opt_update_grid : 1024;
  const bool timed = ctx->opt_time_update != 0;
  ctx->last_update_ms = 0.0;
  ctx->last_launches = 0;
  ctx->last_flips = 0;
  const int nupd = max_np + (pend ? 1 : 0);   // update launches per sweep
  if (timed && ctx->tev.size() < static_cast<size_t>(2 * nupd)) {
    for (hipEvent_t ev : ctx->tev) hipEventDestroy(ev);
    ctx->tev.assign(2 * nupd, nullptr);
    for (auto &ev : ctx->tev) HIP_TRY(ctx, hipEventCreate(&ev));
  }
  std::vector<unsigned long long> chg0;
  if (timed) {
    chg0.resize(4 * static_cast<size_t>(ctx->n_chains));
    HIP_TRY(ctx, hipMemcpy(chg0.data(), ctx->blk_prop, chg0.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  }
  // a block sweep starts and ends without pending moves (the delayed single-link updates
  // share U and rcnt)
  if (pend) ggf_block_pending_launch(bl, false, s);
  for (int sw = 0; sw < n_sweeps; ++sw) {
    for (int p = 0; p < max_np; ++p) {
      bl.patch = p;
      bl.parity = p & 1;
      ggf_block_decide_launch(bl, s);
      if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2 * p], s));
      ggf_block_update_launch(bl, grid, s);
      if (pend) ggf_block_merge_launch(bl, s);
      if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2 * p + 1], s));
    }
    if (pend && max_np > 0) {
      // apply every pending move; the last decision cleared counter max_np & 1
      bl.parity = max_np & 1;
      ggf_block_pending_launch(bl, true, s);
      if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2 * max_np], s));
      ggf_block_update_launch(bl, grid, s);
      if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2 * max_np + 1], s));
      ggf_block_pending_launch(bl, false, s);
    }
    ggf_launch_end_sweep(bl.lc);
    HIP_TRY(ctx, hipGetLastError());
    if (timed) {
      HIP_TRY(ctx, hipStreamSynchronize(s));
      for (int p = 0; p < nupd; ++p) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->tev[2 * p], ctx->tev[2 * p + 1]));
        ctx->last_update_ms += ms;
      }
      ctx->last_launches += nupd;
    }
    if ((st = after_sweep(ctx, s)) != GGF_OK) return st;
  }
  if (timed) {
    std::vector<unsigned long long> chg1(chg0.size());
    HIP_TRY(ctx, hipMemcpy(chg1.data(), ctx->blk_prop, chg1.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (int c = 0; c < ctx->n_chains; ++c) ctx->last_flips += static_cast<long long>(chg1[4 * c + 2] - chg0[4 * c + 2]);
  }
  return GGF_OK;
}

ggf_status ggf_block_stats(ggf_ctx *ctx, int32_t chain, uint64_t *proposals, uint64_t *accepts,
                           uint64_t *links_changed, uint64_t *updates) {
  if (!ctx) return GGF_EINVAL;
  if (chain < 0 || chain >= ctx->n_chains) return fail(ctx, GGF_EINVAL, "chain index out of range");
  HIP_TRY(ctx, hipDeviceSynchronize());
  uint64_t v[4] = {0, 0, 0, 0};
  if (ctx->blk_prop)
    HIP_TRY(ctx, hipMemcpy(v, ctx->blk_prop + 4 * chain, sizeof(v), hipMemcpyDeviceToHost));
  if (proposals) *proposals = v[0];
  if (accepts) *accepts = v[1];
  if (links_changed) *links_changed = v[2];
  if (updates) *updates = v[3];
  return GGF_OK;
}

ggf_status ggf_stream_probe(int32_t mode, void *a, void *b, size_t bytes, int32_t grid, void *stream) {
  const bool needs_b = mode < 2 || mode == 4 || mode >= 6;
  if (!a || (needs_b && !b) || bytes % 16 != 0 || grid < 0 || mode < 0 || mode > 7) return GGF_EINVAL;
  if (ggf_launch_probe(mode, a, b, bytes, grid ? grid : 4096, static_cast<hipStream_t>(stream)) != 0)
    return GGF_EINVAL;
  return hipGetLastError() == hipSuccess ? GGF_OK : GGF_EDEVICE;
}

const char *ggf_last_error(ggf_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

#ifndef GGF_SOURCE_DIGEST
#define GGF_SOURCE_DIGEST "unknown"
#endif
const char *ggf_source_digest(void) { return GGF_SOURCE_DIGEST; }

void ggf_destroy(ggf_ctx *ctx) {
  if (!ctx) return;
  free_chains(ctx);
  for (void *p : ctx->nn_allocs) hipFree(p);
  if (ctx->tensors_dev) hipFree(ctx->tensors_dev);
  for (hipEvent_t ev : ctx->tev) hipEventDestroy(ev);
  if (ctx->ev_in) hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) hipEventDestroy(ctx->ev_out);
  if (ctx->own_stream) hipStreamDestroy(ctx->own_stream);
  delete ctx;
}

}  // extern "C"
