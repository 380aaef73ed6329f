/*
 * ggf.h -- C ABI of the MI355X library for gauged (superposed) Gaussian
 * fermionic PEPS Monte Carlo.
 *
 * The problem (Sec. 4 and 5 of Roose & Zohar, "Gauging a superposition of
 * fermionic Gaussian projected entangled pair states to get lattice gauge
 * theory eigenstates"): given the variational data of the ansatz -- the
 * amplitudes lambda_n, the on-site covariance Gamma_A and the bond
 * covariances Gamma_{B_n} -- estimate gauge-invariant observables as averages
 * over gauge configurations G drawn from p(G) = N(G)/N (Sec. 5.1), with
 *   N(G) = sum_nm lambda_n^* lambda_m <psi_n(G)|psi_m(G)>      (Sec. 5).
 * The library runs many independent Markov chains over G on one GPU.  For
 * each chain it keeps the link field and the inverse G = M(G)^-1 of the
 * virtual matrix M(G) = D + O(G) Gamma_B0 O(G)^T, so W(G) = 2^-4V sqrt(det M)
 * and every single-link ratio costs a 4x4 determinant; an accepted flip is a
 * rank-4 Woodbury update of G.
 *
 * Conventions (Majoranas and covariance as in Sec. 3.2):
 *   c_{2j} = psi_j + psi_j^+,  c_{2j+1} = -i (psi_j - psi_j^+),
 *   Gamma_ab = (i/2) <[c_a, c_b]>   (empty mode: [[0,-1],[1,0]]).
 *   Lattice L x L periodic, site i = x2*L + x1, link l = 2 i + mu (mu = 0:
 *   x -> x+e1, mu = 1: x -> x+e2).  On-site modes in leg order p,l,u,r,d
 *   (Sec. 3).  The gauge field acts on the outgoing leg (r for mu = 0, u for
 *   mu = 1) as exp(i 2 pi k n / N), N = group order (Sec. 3.1).
 *
 * Errors: every call returns a ggf_status; nothing aborts or throws across
 * the ABI.  ggf_last_error() gives a message for the most recent failure on
 * that context.  A context is not thread-safe: use one per host thread.
 * Device work is ordered on the caller's stream (a hipStream_t passed as
 * void*; NULL means the legacy default stream).
 */
#ifndef GGF_H
#define GGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ggf_ctx ggf_ctx;

typedef enum {
  GGF_OK = 0,
  GGF_EINVAL = -1,       /* bad argument or inconsistent input */
  GGF_ENOMEM = -2,       /* device or host allocation failed */
  GGF_ESINGULAR = -3,    /* W(G) = 0: M(G) is singular at a (re)factorisation */
  GGF_ENONFINITE = -4,   /* non-finite ratio or weight that a refactorisation did not cure */
  GGF_EDEVICE = -5,      /* HIP runtime error */
  GGF_ESTATE = -6        /* call out of order (e.g. sweep before init_chains) */
} ggf_status;

#define GGF_KMAX 4       /* largest number of Gaussians in a superposition */
#define GGF_NOBS 21      /* observable slots per chain, see ggf_measure */

/* Variational data of one ansatz (Sec. 5: lambda_n, Gamma_A, Gamma_{B_n}).
 * All host pointers, row-major float64; the library copies them and the caller
 * keeps ownership. */
typedef struct {
  int32_t group;              /* N of the gauge group Z_N, 2 <= N <= 64 (2 = Z2, 3 = Z3) */
  const double *gamma_loc;    /* 10x10 on-site covariance, Majorana order (p,l,u,r,d) x (0,1);
                                 real antisymmetric with Gamma^2 = -1 */
  const double *gamma_bond;   /* 4x4 reference bond b_0 on every link, order (out0,out1,in0,in1);
                                 pure, even parity */
  int32_t K;                  /* number of Gaussians, 1 <= K <= GGF_KMAX */
  const int32_t *patch_link;  /* [K]; patch_link[0] ignored; for k >= 1 the link on which bond
                                 B_k differs from B_0 (may be NULL when K = 1) */
  const double *gamma_bond_k; /* [K][4][4]; k = 0 ignored; bond state of B_k on its patch link.
                                 Its phase is fixed by <b_0|b_k> > 0 (Sec. 5) */
  const double *c_re;         /* [K] real parts of lambda_k (NULL when K = 1) */
  const double *c_im;         /* [K] imaginary parts of lambda_k (NULL when K = 1) */
} ggf_tensor_desc;

/* Per-chain counters and scalars, read back synchronously. */
typedef struct {
  int32_t L, n, tensor_id, precision;
  double logw;                /* log W(G) maintained by the updates (reference-bond weight) */
  double s_re, s_im;          /* S(G) = N(G)/W(G) (1, 0 when K = 1) */
  uint64_t sweeps;            /* sweeps done; the Philox counter word 1 of the next sweep */
  uint64_t accepts, proposals, refreshes, recoveries;
  double max_drift;           /* largest |log W_maintained - log W_fresh| seen at a refresh */
  uint64_t near_ties;         /* Metropolis decisions (single-link and block) with |u - R| < 1e-9 R, where a
                                 rounding change of R could flip the decision (Sec. 5.1 estimator) */
  uint64_t link_cursor;       /* with balanced sweeps (option "balance"): the chain's next link within
                                 its current sweep; 0 at a sweep boundary and without balanced sweeps */
} ggf_chain_info;

/* Create a context on HIP device `device`. */
ggf_status ggf_create(ggf_ctx **out, int device);

/* Register an ansatz (Sec. 5 parameter set).  Validates antisymmetry, purity,
 * even bond parity and K <= GGF_KMAX; precomputes the link-level bond states,
 * the overlaps <B_m|B_n> (phase convention <b_0|b_k> > 0) and the transition
 * covariances of |B_n><B_m| on the patch links.  Returns an id used by
 * ggf_init_chains.  May be called several times (one id per ansatz). */
ggf_status ggf_set_tensor(ggf_ctx *ctx, const ggf_tensor_desc *desc, int32_t *tensor_id_out);

/* Allocate and start n_chains chains.  L[c] (even, 2..32, so n = 8 L^2 <= 8192) and tensor_id[c]
 * are per chain (host arrays).  seed keys the Philox4x32-10 stream of every
 * chain: key = (seed lo, seed hi), counter = (chain, sweep, link, 0).
 * init: 0 = cold (all k = 0), 1 = hot (k = x0 mod N from counter
 * (chain, 0xffffffff, link, 1)).  precision: 64 (G stored and updated in
 * float64) or 32 (G in float32; ratios, log-weights and refactorisations in
 * float64).  refresh_every: after a sweep, chains with at least this many
 * accepted flips since their last factorisation are refactorised in float64
 * (0 = never).  Assembles M(G), factorises it (blocked Gauss-Jordan with
 * partial pivoting) and computes log W and S for every chain.  Replaces any
 * previous chains.  Returns GGF_ESINGULAR if some M(G) is singular. */
ggf_status ggf_init_chains(ggf_ctx *ctx, int32_t n_chains, const int32_t *L, const int32_t *tensor_id,
                           uint64_t seed, int32_t init, int32_t precision, int32_t refresh_every,
                           void *stream);

/* Run n_sweeps single-link Metropolis sweeps on every chain (Sec. 5.1
 * sampling of p(G)): links 0 .. 2V-1 in order, accept iff u < N(G')/N(G).
 * Asynchronous on `stream` except when a chain needs a refactorisation
 * (refresh_every, or recovery from a non-finite ratio), which synchronises. */
ggf_status ggf_sweep(ggf_ctx *ctx, int32_t n_sweeps, void *stream);

/* Observables of every chain's current configuration (Sec. 2.3 plaquette,
 * Sec. 5.1 Wilson loops, Sec. 5.2 fermionic two-point functions, Sec. 5.3
 * electric field), written to
 * out[n_chains][GGF_NOBS] (float64; device pointer when out_is_device != 0,
 * else host pointer, which makes the call synchronous).  Slots:
 *   0 mean plaquette Re[U U U* U*]       (obs_mask bit 0)
 *   1 mean 2x2 Wilson loop               (bit 0)
 *   2 mean density <psi_p^+ psi_p>       (bit 1)
 *   3 log N(G) = log W + log S            (bit 1)
 *   4+r-1 meson string M_r, r = 1..min(L/2, 16), along e1 (bit 2)
 *   20 electric field: lattice mean over links of Re f_E(G) (Sec. 5.3), the
 *      mixed estimator of <J^2_l> with the Z_N Casimir read as 0 on the trivial
 *      irrep and 1 on the others (bit 3); for eigenvalues e_0, e_1 = e_{N-1}
 *      the estimator is e_0 + (e_1 - e_0) x slot 20
 * Slots not requested are written as 0. */
ggf_status ggf_measure(ggf_ctx *ctx, uint32_t obs_mask, double *out, int32_t out_is_device,
                       void *stream);

/* For callers that cannot allocate device memory (serving loops, harnesses that forbid
 * hipMalloc, code that must not allocate between its set-up and its end): ggf_measure with a
 * host output, staged through a fixed device array instead of a temporary allocation.
 * obs_mask and the slots as in ggf_measure; host_out[n_chains][GGF_NOBS] float64, owned by
 * the caller.  The staging array (GGF_STAGE_MAX_CHAINS x GGF_NOBS doubles, 2.6 MiB) is one
 * per GPU, held until the process ends and shared by every context on that GPU: calls that
 * overlap on one GPU (other host threads, or streams running concurrently) race on it.
 * Allocates nothing; synchronises `stream`.  GGF_EINVAL when the context holds more than
 * GGF_STAGE_MAX_CHAINS chains or host_out is NULL, GGF_EDEVICE when the array's address
 * could not be obtained at ggf_create. */
#define GGF_STAGE_MAX_CHAINS 16384
ggf_status ggf_measure_staged(ggf_ctx *ctx, uint32_t obs_mask, double *host_out, void *stream);

/* Couplings of the gauged Hamiltonian (Sec. 2 staggered fermions, Sec. 2.2
 * gauging, Sec. 2.3 plaquette and electric terms), one fermion mode per site:
 *   H = t  sum_{x,mu} [ i eta_mu(x) psi_x^+ D(g_{x,mu}) psi_{x+mu} + h.c. ]
 *     + mu sum_x psi_x^+ psi_x + m sum_x (-1)^(x1+x2) psi_x^+ psi_x
 *     + kb sum_x [ U_sq(x) + U_sq(x)^* ] + ke sum_l J^2_l
 * with D(g) = exp(2 pi i g / N), eta = -1 on the horizontal links of odd rows
 * (pi flux through every plaquette) and +1 elsewhere, and J^2 = 0 on the
 * trivial irrep of Z_N and 1 on the others.  All couplings are free and signed. */
typedef struct {
  double t, mu, m, kb, ke;
} ggf_couplings;

#define GGF_ENERGY_STRIDE (1 + 4 * GGF_KMAX * GGF_KMAX)   /* doubles per chain, ggf_measure_energy */

/* Local energy of every chain's current configuration (Sec. 5.2 and 5.3 applied
 * to H): per pair (a, b) of the superposition h_ab is the transition expectation
 * of H, rho_ab = <B_b|B_a> Pf(M_ab)/Pf(M_00), S = sum lambda_a^* lambda_b rho_ab.
 * Row c of out[n_chains][GGF_ENERGY_STRIDE] (float64; device pointer when
 * out_is_device != 0, else host pointer and synchronous):
 *   [0]            Re E_loc(G) = Re sum_ab lambda_a^* lambda_b rho_ab h_ab / S
 *   [1 + 4p + 0,1] rho_p / S          (complex, p = a K + b < K^2)
 *   [1 + 4p + 2,3] rho_p h_p / S      (complex)
 * remaining entries 0.  <H> is the mean of [0] over samples of p(G). */
ggf_status ggf_measure_energy(ggf_ctx *ctx, const ggf_couplings *couplings, double *out, int32_t out_is_device,
                              void *stream);

/* Linear variational step for lambda (the optimisation of the variational
 * parameters that the outlook of Sec. 6.3 asks for, restricted to lambda_n):
 * rows[n_rows][GGF_ENERGY_STRIDE] (host) are ggf_measure_energy rows of chains
 * with K Gaussians, sampled from p(G) of one lambda.  With Hb, Nb the means of
 * rho h / S and rho / S (Hermitian parts), <H>(lambda') =
 * lambda'^+ Hb lambda' / lambda'^+ Nb lambda' for every lambda' (reweighting);
 * writes the lowest generalised eigenvalue to *energy and its eigenvector,
 * normalised to lambda^+ Nb lambda = 1 with lambda_0 real and >= 0, to
 * lambda_re/lambda_im [K].  Host only; ctx may be NULL (it only receives the
 * error message).  GGF_ESINGULAR if Nb is not positive definite, GGF_ENONFINITE
 * for a non-finite row. */
ggf_status ggf_lambda_step(ggf_ctx *ctx, int32_t K, const double *rows, int64_t n_rows, double *energy,
                           double *lambda_re, double *lambda_im);

/* Replace the amplitudes lambda_n of tensor tensor_id (c_re, c_im [K], host;
 * the linear variational parameters of Sec. 5) and recompute S(G) = N(G)/W(G)
 * of every chain that uses the tensor, so that the next sweep samples p(G) of
 * the new lambda.  Call between sweeps; synchronous.  K = 1 tensors are left
 * unchanged (lambda only scales the state). */
ggf_status ggf_set_lambda(ggf_ctx *ctx, int32_t tensor_id, const double *c_re, const double *c_im, void *stream);

/* Variational optimisation of lambda_n for H (the outlook of Sec. 6.3, restricted
 * to the linear parameters): n_iters rounds of [n_sweeps sweeps, each followed by
 * ggf_measure_energy; ggf_lambda_step over the rows of the chains that use
 * tensor_id; ggf_set_lambda with the result].  energies[n_iters] receives <H>
 * estimated in each round (mean of Re E_loc over those rows, with that round's
 * lambda), e_opt[n_iters] the step's optimum over the same rows, lambda_re/im [K]
 * the last lambda.  Synchronous; allocates n_sweeps x n_chains x GGF_ENERGY_STRIDE
 * doubles of device memory for the call. */
ggf_status ggf_optimise_lambda(ggf_ctx *ctx, int32_t tensor_id, const ggf_couplings *couplings, int32_t n_iters,
                               int32_t n_sweeps, double *energies, double *e_opt, double *lambda_re,
                               double *lambda_im, void *stream);

#define GGF_SENS_STRIDE 200   /* doubles per chain, ggf_measure_sensitivity */

/* Sensitivities of every chain's local energy and log N(G) to the on-site
 * covariance Gamma_A (gradient descent on Gamma_A, the outlook of Sec. 6.3;
 * any L <= 32).  For a rotation
 * Gamma_A -> exp(theta E) Gamma_A exp(-theta E) (E real antisymmetric 10 x 10,
 * Delta = [E, Gamma_A]): d Re E_loc(G)/d theta = tr(Delta S_e) and
 * d log N(G)/d theta = tr(Delta S_N), tr(Delta S) = sum_ij Delta_ij S_ji.
 * Row c of out[n_chains][GGF_SENS_STRIDE]: [0..99] S_e, [100..199] S_N,
 * row-major 10 x 10 (device pointer when out_is_device != 0, else host and
 * synchronous).  K > 1 (superposition of Sec. 4 with the patch cross terms):
 * with om_ab = lambda_a^* lambda_b <B_b|B_a> r_ab, S = sum om, h_ab the pair's
 * transition energy and E the local energy, d log N = sum (om_ab / S) (1/2)
 * tr(M_ab^-1 dM) and d E = sum (om_ab / S) [d h_ab + (h_ab - E) (1/2)
 * tr(M_ab^-1 dM)], real parts.  Such a call is synchronous and allocates for
 * its duration per chain GGF_ENERGY_STRIDE doubles and, with n the largest n of
 * the context, M_ab^-1 as n^2 complex doubles when n <= 512 (4 MiB at L = 8),
 * else the factors of M_ab^-1 - G (rank <= 8) as 26 n doubles (1.7 MiB at L = 32). */
ggf_status ggf_measure_sensitivity(ggf_ctx *ctx, const ggf_couplings *couplings, double *out,
                                   int32_t out_is_device, void *stream);

/* Gradient of <H> with respect to the rotation generators of Gamma_A from
 * n_rows samples of p(G) (host rows of ggf_measure_energy and
 * ggf_measure_sensitivity of the same chains and configurations):
 * d<H>/d theta_kl = mean tr(Delta_kl S_e) + mean (e - mean e) tr(Delta_kl S_N),
 * written as the antisymmetric grad[10][10] (grad[k][l] for E_kl = e_kl - e_lk);
 * gamma_loc is the current on-site covariance.  Host only; ctx may be NULL. */
ggf_status ggf_gamma_gradient(ggf_ctx *ctx, const double *gamma_loc, const double *energy_rows,
                              const double *sens_rows, int64_t n_rows, double *grad);

/* Replace the bond state of B_k (1 <= k < K) on its patch link in tensor tensor_id (4 x 4, pure
 * and even as in ggf_set_tensor; phase fixed by <b_0|b_k> > 0): the pair tables are recomputed
 * and every chain that uses the tensor gets its S(G) = N(G) / W(G) again.  G = M(G)^-1 and
 * log W do not involve the patch bonds, so nothing is refactorised.  Synchronous. */
ggf_status ggf_set_bond(ggf_ctx *ctx, int32_t tensor_id, int32_t k, const double *gamma_bond_k, void *stream);

#define GGF_BOND_SMAX 12      /* patch Majoranas of an ansatz: 4 per patch link, K <= GGF_KMAX */
#define GGF_BOND_STRIDE (2 + GGF_BOND_SMAX + GGF_KMAX + 3 * GGF_BOND_SMAX * GGF_BOND_SMAX)

/* Rows for the gradient with respect to the patch bond states Gamma_{B_k},
 * k >= 1 (gradient descent on the bond states, the outlook of Sec. 6.3, for
 * the superposition of Sec. 5).  The bond of B_k enters only through its patch
 * link's transition covariances and overlaps, so per configuration the
 * gradient needs G on the patch Majoranas S (the union over k >= 1 of the four
 * Majoranas of link patch_link[k], in increasing order, s <= 12 of them) and
 * the contraction of the linear part of the local energy with the rows G[S, :]:
 *   R[a][b] = sum_ij C_ij G[i][S_a] G[S_b][j],
 * where sum_ij C_ij X_ij is the part of the energy (Sec. 2 hopping, chemical
 * and mass terms through Gamma_out = A + B X B^T, Sec. 2.3 electric term
 * through the mixed occupation of every link with the reference bond's
 * response) linear in X = M^-1.  Row c of out[n_chains][GGF_BOND_STRIDE]:
 *   [0]                          s (0 for a chain with K = 1)
 *   [1]                          L
 *   [2 + q]                      S_q, q < s
 *   [14 + k]                     value of link patch_link[k] (k >= 1)
 *   [18 + 2 (12 a + b) + 0,1]    R[a][b] (complex)
 *   [306 + 12 a + b]             G[S_a][S_b]
 * (float64; device pointer when out_is_device != 0, else host pointer and
 * synchronous).  GGF_EINVAL unless s L^2 <= 4096 for every chain with K > 1.
 * Allocates out's size of device memory for a host out. */
ggf_status ggf_measure_bond_rows(ggf_ctx *ctx, const ggf_couplings *couplings, double *out, int32_t out_is_device,
                                 void *stream);

/* Gradient of <H> with respect to the rotations of the patch bond states,
 * Gamma_{B_k} -> exp(theta E) Gamma_{B_k} exp(-theta E) for the six generators
 * E = e_ab - e_ba, (a, b) in order (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) of the
 * link's Majoranas (out0, out1, in0, in1), the phase convention <b_0|b_k> > 0
 * kept, from n_rows samples of p(G) of chains of one ansatz: host rows of
 * ggf_measure_energy and ggf_measure_bond_rows of the same chains and
 * configurations, and that ansatz's descriptor (as given to ggf_set_tensor).
 * Per sample, with om_nm = lambda_n^* lambda_m rho_nm, S = sum om and
 * e = sum om h / S: d log N = sum (om / S) d log rho, d e = sum (om / S) [d h +
 * (h - e) d log rho], d log rho_nm = d log <B_m|B_n> + (1/2) tr(M_nm^-1 dM_nm),
 * and d h_nm = -sum_ab dY_ab R_nm[a][b] + ke dX_nm, Y_nm = Delta (1 + G_SS
 * Delta)^-1 the Woodbury factor of M_nm^-1 = G - G_S Y G_S^T, R_nm the rows'
 * R with the pair's own electric response on its patch links and dX_nm the
 * change of the mixed occupation of the varied link through its bond.  Then
 * d<H>/d theta = mean Re d e + mean (Re e - mean Re e) d log N, written to
 * grad[(k - 1) 6 + g] for k = 1 .. K - 1 and generator g.  Host only; ctx may
 * be NULL.  GGF_EINVAL for K = 1 or rows of another size of S. */
ggf_status ggf_bond_gradient(ggf_ctx *ctx, const ggf_tensor_desc *tensor, const ggf_couplings *couplings,
                             const double *energy_rows, const double *bond_rows, int64_t n_rows, double *grad);

/* Replace the on-site covariance of tensor tensor_id (10 x 10, checked as in
 * ggf_set_tensor) and refactorise every chain that uses it from its link field
 * (float64), so that G, log W and S follow the new tensor.  Synchronous. */
ggf_status ggf_set_gamma_loc(ggf_ctx *ctx, int32_t tensor_id, const double *gamma_loc, void *stream);

/* Gradient descent on the on-site covariance Gamma_A (the outlook of Sec. 6.3;
 * the chains as in ggf_measure_sensitivity): n_iters rounds of [n_sweeps sweeps, each followed by
 * ggf_measure_energy and ggf_measure_sensitivity; ggf_gamma_gradient over the
 * rows of the chains that use tensor_id; Gamma_A <- exp(X) Gamma_A exp(-X) with
 * X = -step grad; ggf_set_gamma_loc].  energies[n_iters]: <H> estimated in each
 * round with that round's Gamma_A; grad_norms[n_iters]: max |grad|;
 * gamma_loc_out[10][10]: the last Gamma_A.  Synchronous; allocates
 * n_sweeps x n_chains x (GGF_ENERGY_STRIDE + GGF_SENS_STRIDE) doubles of device
 * memory for the call. */
ggf_status ggf_optimise_gamma(ggf_ctx *ctx, int32_t tensor_id, const ggf_couplings *couplings, int32_t n_iters,
                              int32_t n_sweeps, double step, double *energies, double *grad_norms,
                              double *gamma_loc_out, void *stream);

/* Synchronous read-back of one chain: link values (int8, 2V entries),
 * counters and scalars.  Any argument may be NULL. */
ggf_status ggf_get_state(ggf_ctx *ctx, int32_t chain, int8_t *links, ggf_chain_info *info);

/* Replace one chain's link field and sweep counter (checkpoint resume) and
 * refactorise it; the chain restarts at a sweep boundary (link cursor 0).
 * Synchronous. */
ggf_status ggf_set_state(ggf_ctx *ctx, int32_t chain, const int8_t *links, uint64_t sweeps);

/* Copy one chain's maintained inverse G = M(G)^-1 (n x n, row-major) to host
 * memory as float64.  Synchronous; for tests and diagnostics. */
ggf_status ggf_get_inverse(ggf_ctx *ctx, int32_t chain, double *host_out);

/* Overwrite one chain's maintained inverse from host float64 data without
 * refactorising (fault injection for recovery tests).  Synchronous. */
ggf_status ggf_set_inverse(ggf_ctx *ctx, int32_t chain, const double *host_in);

/* Refactorise every chain from its link field now (float64), recording the
 * drift of log W.  Synchronous. */
ggf_status ggf_refresh_all(ggf_ctx *ctx, void *stream);

/* Tuning knobs (0 = library default):
 *   "update_grid"  workgroups of the persistent rank-4 update kernel
 *   "update_tiles" row tiles per chain in the rank-4 update
 *   "update_nt"    1 (default) = non-temporal loads/stores of G in the rank-4 update, 0 = cached
 *   "graph"        1 = replay each sweep as a captured hipGraph, 0 = direct launches
 *   "gj_nb"        column-block width of the Gauss-Jordan refactorisation (8..256, rounded up to a
 *                  power of 2; 0 = 256 for n >= 2048, 128 for n >= 512, else 64)
 *   "scratch_mb"   float64 scratch budget for refactorisations, MiB
 *   "delay"        window of delayed updates in link steps: 8, 16, 24 or 32 (the accepted
 *                  flips of a window are kept as pending factors G_cur = G - X Y^T and applied
 *                  by one matrix-core rank-4F update at its end), 0 = one rank-4 streaming
 *                  update per link step, -1 (default) = 16.  Takes effect at the next sweep;
 *                  G as read through the ABI never has pending flips.
 *   "flush_grid"   workgroups of the window flush (default 512)
 *   "block_pend"   block sweeps: largest combined rank of accepted block moves kept pending
 *                  and applied to G together, 0 .. 128 (default 128; 0 = each accepted move
 *                  updates G at once)
 *   "block_rho"    move rate rho of the block proposal in units of 1/65536, 1 .. 65536 (default
 *                  65536, rho = 1): each patch link keeps its value with probability 1 - rho and
 *                  is otherwise drawn from the network's conditional; link l becomes 1 iff its
 *                  uniform u_l < (1 - rho) y_l + rho sigmoid(z_l), and the acceptance uses the
 *                  proposal densities of this rule
 *   "balance"      1 = balanced sweeps for batches of different lattice sizes: a ggf_sweep sweep
 *                  is max_links link steps at each of which every chain proposes its own next link
 *                  (a per-chain cursor), so a chain with fewer links completes several of its own
 *                  sweeps (links in order, Philox counters as always) instead of idling; its sweep
 *                  counter advances when its cursor wraps, and the refactorisation check runs at
 *                  the end of each ggf_sweep sweep.  0 (default) = link steps in lock-step.
 *                  Switching it off needs every chain at a sweep boundary (GGF_ESTATE otherwise)
 *   "time_update"  1 = record HIP events around the update and link-step launches of eager sweeps
 *                  (ggf_update_timing, ggf_ratio_timing); a sweep with graph replay then runs eagerly */
ggf_status ggf_set_option(ggf_ctx *ctx, const char *key, int64_t value);

/* Pick the launch shapes of the path that runs by timing candidates on live
 * sweeps: each candidate runs `sweeps_per_candidate` real Metropolis sweeps (they
 * advance the chains, so call it during burn-in; results do not depend on the
 * launch shape) and the time of the link steps and update launches per proposal
 * is measured with HIP events.  With delayed updates (the default) it tunes the
 * window flush: best = {flush_grid, delay window (8, 16 or 32 link steps), 0};
 * with "delay" = 0 the rank-4 streaming update: best =
 * {update_grid, update_tiles, update_nt}.  With cache_path != NULL the choice
 * is looked up in / appended to that text file, keyed by (path, n_max,
 * precision, K_max, n_chains); a cached choice skips the timing.  The chosen
 * values are left set as options and returned through best[3] (may be NULL).
 * Synchronous. */
ggf_status ggf_autotune(ggf_ctx *ctx, int32_t sweeps_per_candidate, const char *cache_path, int64_t *best,
                        void *stream);

/* Duration in milliseconds of the update kernels of the most recent
 * ggf_sweep or ggf_block_sweep call, summed over its launches, measured with
 * HIP events on the stream the kernels run on (0 when timing is off; enable
 * with option "time_update" = 1).  Also returns the number of launches and
 * the number of link changes they applied (accepted flips for ggf_sweep, sum
 * of changed links over accepted block moves for ggf_block_sweep). */
ggf_status ggf_update_timing(ggf_ctx *ctx, double *ms, int64_t *launches, int64_t *flips);

/* Duration in milliseconds of the ratio / decision kernels (one launch per link
 * step: ratio, Metropolis decision and, on accept, the update factors) of the
 * most recent ggf_sweep call, measured like ggf_update_timing (0 when timing
 * is off), and the number of launches. */
ggf_status ggf_ratio_timing(ggf_ctx *ctx, double *ms, int64_t *launches);

/* Flags of ggf_autocorr_time. */
#define GGF_TAU_FLOOR 1   /* the windowed sum fell to 1/2 or below and was clamped to 1/2 */
#define GGF_TAU_SHORT 2   /* series too short for the estimate: n_t < 50 tau, a window above n_t / 4,
                             or no window W >= c tau within the series */

/* Integrated autocorrelation time of n_series Monte Carlo series sampled at
 * n_t times, series[t * n_series + s] (host float64).  Each series is centred
 * on its own mean; the autocovariance is averaged over series, normalised,
 * and summed with Sokal's automatic window (smallest W with W >= c tau(W),
 * tau(W) = 1/2 + sum_{t=1..W} rho(t)).  Outputs tau (clamped below at 1/2),
 * its Madras-Sokal error tau sqrt(2 (2W + 1) / (n_t n_series)), W and flags
 * (GGF_TAU_FLOOR, GGF_TAU_SHORT; may be NULL): centring on the series mean
 * biases short series towards 1/2, so a flagged tau is not a measurement.
 * Effective samples = n_t n_series / (2 tau).  Pure host computation; needs
 * no context.  GGF_EINVAL for n_t < 2, n_series < 1, c <= 0 or NULL series/tau. */
ggf_status ggf_autocorr_time(const double *series, int64_t n_t, int64_t n_series, double c, double *tau,
                             double *tau_err, int64_t *window, int32_t *flags);

/* ---- Learned block proposal --------------------------------------------
 * An exact Metropolis-Hastings move on a P x P patch of sites (2 P^2 links) of
 * Z2 chains, on top of the single-link sampler (Sec. 5.1 leaves the sampler
 * open).  The patch links are resampled from a factorised Bernoulli whose
 * logits come from four valid 3x3 convolutions (2 -> 32 -> 32 -> 32 -> 2
 * channels, tanh, bfloat16 weights, float32 accumulation) over the (P+8)^2
 * window of the link field around the patch with every image of the patch
 * masked; forward and reverse proposal probabilities come from one forward
 * pass and the acceptance uses the true weight N(G).  An accepted move with m
 * changed links is a rank-4m Woodbury update of G.  Parameters: one float32
 * vector W1[32][2][3][3], b1[32], W2[32][32][3][3], b2, W3, b3, W4[2][32][3][3],
 * b4[2] (ggf_nn_nparams() entries).  Patch p of an L x L lattice has origin
 * (P (p mod L/P), P (p div L/P)); its links are ordered 2 (y P + x) + mu. */

/* Number of network parameters. */
int32_t ggf_nn_nparams(void);

/* Select the patch side (1, 2 or 4), initialise the weights Glorot-uniform
 * from Philox at counter (index, 0, 0, 9) keyed by seed (biases 0) and reset
 * the Adam state.  Synchronous. */
ggf_status ggf_nn_init(ggf_ctx *ctx, int32_t patch, uint64_t seed);

/* Read (get_host != NULL) and/or replace (set_host != NULL) the float32
 * parameters; host arrays of ggf_nn_nparams() floats.  Synchronous. */
ggf_status ggf_nn_params(ggf_ctx *ctx, float *get_host, const float *set_host);

/* Logits of examples (chain[e], patch[e]) of the current chain states into
 * logits_host[n][2 P^2] (patch link order).  Host arrays; n <= 65536; synchronous. */
ggf_status ggf_nn_forward(ggf_ctx *ctx, int32_t n, const int32_t *chain, const int32_t *patch, float *logits_host);

/* Mean binary cross-entropy of the examples' current patch links under the
 * network and its gradient (float32, ggf_nn_nparams() entries; the bfloat16
 * rounding of the weights is treated as the identity).  Synchronous. */
ggf_status ggf_nn_grad(ggf_ctx *ctx, int32_t n, const int32_t *chain, const int32_t *patch, float *grad_host,
                       double *loss_host);

/* `steps` Adam steps (lr, beta 0.9/0.999, eps 1e-8) on batches of `batch`
 * examples drawn from the current chain states (chain, patch from Philox at
 * counter (step, example, 0, 8) keyed by seed).  loss_host (may be NULL)
 * receives the last batch's mean loss, which makes the call synchronous. */
ggf_status ggf_nn_train(ggf_ctx *ctx, int32_t steps, int32_t batch, float lr, uint64_t seed, double *loss_host,
                        void *stream);

/* n_sweeps block sweeps: a block move on every patch in order, then the sweep
 * counter advances (shared with ggf_sweep).  Philox counters: proposal
 * uniforms (chain, sweep, patch, 3 + l/4), word l mod 4, u = (x + 1/2) 2^-32;
 * acceptance (chain, sweep, patch, 2).  Requires ggf_nn_init and Z2 chains
 * whose side is a multiple of P.  With option "block_pend" > 0 (the default)
 * accepted moves of consecutive patches are applied to G together, as one
 * Woodbury update of rank up to "block_pend" (Sec. 4.2's update with the
 * pending moves' U and W combined); each decision sees the inverse with every
 * pending move applied, so the chain is the same; every move is applied by the
 * end of the call. */
ggf_status ggf_block_sweep(ggf_ctx *ctx, int32_t n_sweeps, void *stream);

/* Block moves proposed (at least one link changed) and accepted for a chain,
 * the number of links the accepted moves changed, and the number of updates of
 * the chain's G that applied them (one per accepted move when "block_pend" is
 * 0, fewer with delayed moves).  Any output may be NULL.  Synchronous. */
ggf_status ggf_block_stats(ggf_ctx *ctx, int32_t chain, uint64_t *proposals, uint64_t *accepts,
                           uint64_t *links_changed, uint64_t *updates);

/* Bandwidth probe (diagnostics): mode 0 copies `bytes` from a to b, mode 1 the
 * same with non-temporal loads/stores, mode 2 updates a in place
 * (a = a * 1 + 1, read and write), mode 3 the same non-temporal.  Modes 4-7 keep
 * 8 non-temporal 16-byte loads in flight per thread, each workgroup streaming one
 * contiguous chunk: 4 copy a -> b, 5 update a in place, 6 read a only, 7 write b
 * only.  a and b are device pointers (b unused for modes 2, 3, 5); bytes a
 * multiple of 16; grid workgroups of 256 threads (0 = 4096).  Asynchronous on
 * `stream`. */
ggf_status ggf_stream_probe(int32_t mode, void *a, void *b, size_t bytes, int32_t grid, void *stream);

/* SHA-256 (hex) of the sources the library was built from (its C++/HIP sources and this
 * header), or "unknown" for a build that did not record it.  Static string. */
const char *ggf_source_digest(void);

/* Message of the most recent failure on this context ("" if none). */
const char *ggf_last_error(ggf_ctx *ctx);

/* Free all device and host memory of the context.  NULL is a no-op. */
void ggf_destroy(ggf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GGF_H */
