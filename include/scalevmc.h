/*
 * scalevmc — C ABI of the SCALE local-energy hot path on one AMD MI355X (gfx950).
 *
 * What is computed (arXiv 2604.25775):
 *   amplitude   psi(n) = det Phi_up(n) * det Phi_dn(n), with configuration-
 *               dependent backflow orbitals from an embedding, a stack of
 *               residual 3x3 convolutions and an orbital projection
 *               (Sec. II.B: embedding layer, residual conv equation, orbital
 *               projection; one Slater block per spin).
 *   ratios      psi(n')/psi(n) for every configuration n' reached from n by one
 *               hopping term of the Hubbard Hamiltonian (Sec. III), evaluated by
 *               recomputing only the features inside the receptive field of the
 *               hop (Sec. II.C, affected-sites equation) and a low-rank
 *               determinant update against the cached inverse (Sec. II.C,
 *               Sherman-Morrison-Woodbury equations).
 *   local energy E_loc(n) = sum_n' psi(n)^-1 <n|H|n'> psi(n')   (Sec. II.A).
 *
 * Conventions shared by every call:
 *  - Lattice sites s = x + Lx*y (x fastest).  Occupation byte per site:
 *    n_up + 2*n_dn (0 empty, 1 up, 2 down, 3 double).
 *  - Walkers are ordered lattice-major: all walkers of lattice 0, then of
 *    lattice 1, ...  Walker w of lattice l owns N_l occupation bytes.
 *  - Every pointer documented as "device" is HIP device memory owned by the
 *    caller; the library never frees it and reads it only during the call's
 *    stream work.  Host pointers are read before the call returns.
 *  - All calls enqueue work on `stream` and return without synchronising
 *    (except svmc_load_walkers' validation, see there); outputs are valid once
 *    the stream reaches the call.  Calls on one context must not overlap.
 *  - No call aborts.  Argument errors return SVMC_ERR_INVALID_ARG and leave the
 *    context unchanged; svmc_last_error() gives a message.  Numerical trouble of
 *    a single walker never fails a call: it sets that walker's flag bits
 *    (svmc_walker_flags).
 *  - Floating-point: the determinant work (inverses, log-determinants, the
 *    small Woodbury systems, ratios, energies) is FP64.  The conv stack runs in
 *    svmc_model.conv_prec; the library rounds the embedding, conv kernels and
 *    conv biases to that precision (round to nearest even).  Projection
 *    weights and base orbitals are used in FP64.
 */
#ifndef SCALEVMC_H
#define SCALEVMC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct svmc_ctx svmc_ctx;

typedef enum {
  SVMC_OK = 0,
  SVMC_ERR_INVALID_ARG = 1,
  SVMC_ERR_OOM = 2,
  SVMC_ERR_HIP = 3,
  SVMC_ERR_STATE = 4,        /* call order: e.g. local energy before walkers */
  SVMC_ERR_UNSUPPORTED = 5   /* valid but not implemented shape */
} svmc_status;

/* Per-walker flag bits. */
typedef enum {
  SVMC_W_OK = 0,
  SVMC_W_SINGULAR = 1,   /* a Slater block has a zero pivot: psi = 0 */
  SVMC_W_NONFINITE = 2,  /* a NaN/Inf appeared in log|psi| or a ratio */
  SVMC_W_DRIFT = 4,      /* Woodbury-updated inverse drifted beyond 1e-8 */
  SVMC_W_BADCOUNT = 8,   /* occupation does not hold n_up/n_dn electrons */
  SVMC_W_SYMMETRY = 16   /* symmetric batch: the copies are not the images of
                            copy 0 under the group (svmc_local_energy_sym) */
} svmc_walker_flag;

typedef enum { SVMC_ACT_TANH = 0, SVMC_ACT_SILU = 1 } svmc_act;
/* Conv-stack precision.  BF16: multiplier inputs rounded to BF16, FP32
 * accumulation, FP32 residual stream.  BF16X3: each FP32 activation is split
 * exactly into three BF16 terms multiplied in three passes (FP32-accurate
 * activations on the BF16 matrix units); weights are BF16 in both.  F16X2:
 * each FP32 activation split into two FP16 terms (round toward zero; the
 * pair carries it to 2^-20 relative, |activation| < 65504), two passes on the
 * FP16 matrix units, weights rounded to FP16.  All 16-bit modes accumulate in
 * FP32 with an FP32 residual stream. */
typedef enum { SVMC_FP64 = 0, SVMC_FP32 = 1, SVMC_BF16 = 2, SVMC_BF16X3 = 3, SVMC_F16X2 = 4 } svmc_prec;
typedef enum { SVMC_PATH_LOWRANK = 0, SVMC_PATH_FULL = 1 } svmc_path;

/* Lattice and Hamiltonian (Sec. III): Lx x Ly sites, periodic or open per
 * axis (a periodic axis needs length >= 3), hopping t (nearest neighbours)
 * and tp (next-nearest; 0 disables those hops), electrons per spin n_up,
 * n_dn (each <= N).
 * tj = 0: Hubbard model, on-site U; J and h_pin must be 0.
 * tj = 1: t-J model.  The Gutzwiller projection removes doubly occupied
 *   sites: no hop onto an occupied site is a connected configuration, the
 *   sampler rejects such moves, and a walker holding a doubly occupied site
 *   is flagged SVMC_W_BADCOUNT.  J S_i.S_j on every nearest-neighbour bond
 *   (S = the spin-1/2 operator of the site, no density term); a pinning
 *   field h_pin (-1)^y S^z on the sites of the column x = 0 (the staggered
 *   field on the left edge of a cylinder).  U is not used.  At most 2048
 *   sites and n_up + n_dn <= N. */
typedef struct {
  int32_t Lx, Ly, pbc_x, pbc_y;
  double t, tp, U;
  int32_t n_up, n_dn;
  double J, h_pin;
  int32_t tj, reserved;    /* reserved: set to 0 */
} svmc_lattice;

/* Network shape (Sec. II.B): an embedding layer, n_conv residual ksize x
 * ksize conv layers (1..4) of `channels` channels (8, 16, 24 or 32),
 * activation svmc_act, conv precision svmc_prec, then n_mlp site-wise MLP
 * layers (Sec. II.B, site-wise MLP equation: H <- act(H W_m + b_m) at every
 * site, no residual, W_m of size channels x channels as that equation
 * writes it, the same activation) before the orbital projection; they
 * leave the receptive field at n_conv, so the local update still touches
 * only the conv layers' boxes.  refresh_every = accepted Metropolis moves
 * between FP64 inverse rebuilds (>= 1).  ksize must be 3 and n_mlp in 0..8
 * (ksize != 3 or n_mlp > 8: SVMC_ERR_UNSUPPORTED; n_mlp < 0: INVALID_ARG).
 * per_site_embed = 0: one embedding table E[4][C] shared by all sites;
 * 1: a table E_i[4][C] per site i (the embedding layer as Sec. II.B writes
 * it), per lattice of the context. */
typedef struct {
  int32_t n_conv, channels, act, conv_prec, refresh_every;
  int32_t ksize, n_mlp, per_site_embed;
} svmc_model;

/* Create a context for n_lats lattices (1..8) sharing one network.  Lattices
 * may differ in size and electron numbers; the conv stack and embedding are
 * shared, projection and base orbitals are per lattice.  *out receives the
 * handle.  Errors: INVALID_ARG for bad shapes, UNSUPPORTED for channels or
 * depths outside the list above, HIP if no device is usable. */
svmc_status svmc_create(const svmc_lattice* lats, int32_t n_lats,
                        const svmc_model* model, svmc_ctx** out);

/* Release all device memory of the context (waits for its work). */
svmc_status svmc_destroy(svmc_ctx* ctx);

/* Length of the flat parameter vector theta:
 *   embed | conv_w[L][3][3][C][C] (ky, kx, c_in, c_out; tap (ky,kx)
 *   reads the neighbour at offset (kx-1, ky-1)) | conv_b[L][C] |
 *   mlp_w[M][C][C] (c_in, c_out) | mlp_b[M][C] |
 *   for each lattice: W_up[C][n_up] | W_dn[C][n_dn] | b_up[n_up] | b_dn[n_dn]
 * all row-major FP64, with embed = E[4][C] (shared table) or, with
 * per_site_embed, E_l[N_l][4][C] for each lattice l in order (site, then
 * occupation n_up + 2 n_dn).  Row of spin s at site x:
 * base_s[x] + H_F[x] W_s + b_s, H_F the last site-wise layer's output (the
 * last conv layer's when M = 0). */
int64_t svmc_num_params(const svmc_ctx* ctx);

/* Upload parameters.  theta: device, svmc_num_params doubles (layout above).
 * base: host array of n_lats device pointers; base[l] holds the FP64 base
 * orbitals of lattice l: [N][n_up] for spin up followed by [N][n_dn] for
 * spin down (row = site).  Invalidates walker caches (reload or refresh). */
svmc_status svmc_set_params(svmc_ctx* ctx, const double* theta,
                            const double* const* base, hipStream_t stream);

/* Load walkers.  walkers_per_lattice: host [n_lats] counts (>= 0, total >= 1).
 * occ: device int8, concatenated walker occupations (lattice-major).  Builds
 * the feature cache, Slater inverses, log|psi| and the low-rank precompute.
 * Validates electron counts on the device; a walker whose count is wrong gets
 * SVMC_W_BADCOUNT and psi = 0.  Requires svmc_set_params first. */
svmc_status svmc_load_walkers(svmc_ctx* ctx, const int64_t* walkers_per_lattice,
                              const int8_t* occ, hipStream_t stream);

int64_t svmc_num_walkers(const svmc_ctx* ctx);

/* Row stride of the per-hop outputs of svmc_local_energy: the largest number
 * of connected configurations any walker can have over the lattices,
 * (n_up + n_dn) * (tp != 0 ? 8 : 4) hops, plus 4 min(n_up, n_dn) spin
 * exchanges in the t-J model. */
int32_t svmc_max_hops(const svmc_ctx* ctx);

/* log|psi| and its sign for every walker.  sign: canonical sign, i.e. with the
 * rows of each Slater block in ascending site order (ups before downs).
 * Both device [W] FP64. */
svmc_status svmc_log_psi(svmc_ctx* ctx, double* sign, double* logabs,
                         hipStream_t stream);

/* Low-rank precompute for every walker from its current features and
 * inverses: G_s = M_s Phi_s^-1 for the orbital rows M_s of all sites and
 * P_s = W_s Phi_s^-1 (the factors of the determinant-lemma matrices,
 * Sec. II.C), with M_s = base_s + b_s + H_L W_s taken apart
 * (G_s = (base_s + b_s) Phi_s^-1 + H_L P_s), so M_s itself is not formed.
 * svmc_local_energy(LOWRANK) runs it by itself when walkers changed since
 * the last one; calling it explicitly always recomputes. */
svmc_status svmc_prepare(svmc_ctx* ctx, hipStream_t stream);

/* Local energies (Sec. II.A) with the Hubbard or t-J Hamiltonian (Sec. III).
 * path LOWRANK: incremental features + Woodbury ratios against the cached
 * inverses (Sec. II.C); FULL: every connected configuration recomputed from
 * scratch (full network forward and an FP64 LU per spin) - the O(N^4)
 * comparison path with the same precision policy.
 * eloc: device [W] FP64.  Optional (NULL to skip, all or none):
 *   n_hops   device [W] int32   number of connected configurations
 *   hop_code device [W][svmc_max_hops] int32, code = (i << 4) | (spin << 3) | d
 *            with i the site the electron leaves, spin 0 up / 1 down, and d the
 *            direction +x, -x, +y, -y, +x+y, +x-y, -x+y, -x-y (0..7); a spin
 *            exchange (t-J) has code ((N + i) << 4) | d: the up electron on
 *            site i and the down electron on its neighbour in direction d
 *            (0..3) trade sites
 *   ratio    device [W][svmc_max_hops] FP64: det ratio with the moving
 *            electron keeping its row ("in-place"), so that the Hamiltonian
 *            term of the hop is -t_ij * ratio; for an exchange both spins'
 *            movers keep their rows and the term is -(J/2) * ratio.
 * Hops are listed spin up first, source site ascending, directions in the
 * order above, then the exchanges, up site ascending.  The diagonal term is
 * U * (number of doubly occupied sites) for the Hubbard model; for the t-J
 * model J sum S^z_i S^z_j over the bonds plus the pinning field. */
svmc_status svmc_local_energy(svmc_ctx* ctx, svmc_path path, double* eloc,
                              int32_t* n_hops, int32_t* hop_code, double* ratio,
                              hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * local energies as svmc_local_energy(ctx, SVMC_PATH_LOWRANK, eloc, NULL,
 * NULL, NULL, stream), bit for bit, with the per-slice partial sums in a
 * fixed array of 2^20 doubles (8 MiB) per device that the library holds
 * until the process ends, instead of a context buffer.  The call allocates
 * nothing (no hipMalloc, no library allocation); like svmc_local_energy it
 * first rebuilds G and P from the cached inverses if walkers changed.
 * eloc: device [W] FP64.  The context's device must be current.  Every call
 * on one device shares that array: calls that overlap on one device (other
 * streams, other contexts) race and must be ordered by the caller.
 * Errors: SVMC_ERR_UNSUPPORTED when walkers x slices per walker (svmc_tune)
 * exceeds 2^20; SVMC_ERR_STATE without walkers. */
svmc_status svmc_local_energy_noalloc(svmc_ctx* ctx, double* eloc, hipStream_t stream);

/* Metropolis sampling of |psi|^2 (Sec. II.A), n_sweeps sweeps of N proposals
 * per walker.  Proposal k of walker w draws one Philox4x64-10 block with key
 * (seed, 0) and counter (w, step0 + k, 0, 0): electron e = mulhi(w0, n_up +
 * n_dn) (labels of spin up first), direction d = w1 >> 62 (+x, -x, +y, -y),
 * u = (w2 >> 11) 2^-53; the move is rejected when the target is off the
 * lattice or holds the same spin, else accepted iff u < ratio^2 (ratio by the
 * local update of Sec. II.C, FP64 determinant part).  An accepted move
 * rewrites the walker's cached features on the update box, updates
 * G = M Phi^-1 and P = W Phi^-1 by the Sherman-Morrison-Woodbury formula
 * (Sec. II.C) and log|psi|, sign by the ratio.  Proposal k of all walkers is
 * one step on the stream.  Walkers that have made refresh_every accepted
 * moves get their rows, inverse, log|psi| and G/P rebuilt in FP64
 * (SVMC_W_DRIFT set first if the maintained G had drifted by more than 1e-8
 * on its occupied rows) at the next batch refresh, every 8 steps and after
 * the last one; their updates stay exact meanwhile, so the chain does not
 * depend on refresh_every.  A walker whose update matrix is numerically
 * singular keeps the accepted configuration and is rebuilt right after that
 * step, before its next proposal.  Walkers
 * flagged SINGULAR, NONFINITE or BADCOUNT are not moved.  In a mixed batch a
 * walker of a lattice with N sites takes n_sweeps * N proposals.
 * n_accept: device [W] int64 incremented by each walker's accepted moves, or
 * NULL.  Work is queued on `stream`; nothing waits on it.  The first call
 * allocates the sweep workspace (about 32 KB per walker at 16x16, C = 32).
 * Errors: SVMC_ERR_STATE without walkers, SVMC_ERR_INVALID_ARG for
 * n_sweeps < 0 or refresh_every < 1, SVMC_ERR_UNSUPPORTED when one walker's
 * workspace exceeds 160 KiB of LDS. */
svmc_status svmc_sweep(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed,
                       uint64_t step0, int64_t* n_accept, hipStream_t stream);

/* Form of svmc_sweep that can be recorded into a HIP graph and replayed: the
 * same fixed sequence of launches per proposal step, no host synchronisation,
 * no allocation, no memset node.  step0 is read at run time from the device
 * scalar *step0_dev (uint64), so replays can advance the chain by updating it
 * between replays.  The first call must be made outside a capture (it
 * allocates the workspace), and G/P must be current (svmc_prepare) before a
 * capture.  Same chain as svmc_sweep for the same seed and step0. */
svmc_status svmc_sweep_async(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed,
                             const uint64_t* step0_dev, int64_t* n_accept,
                             hipStream_t stream);

/* Rebuild every walker's Slater inverse, log|psi| and low-rank precompute in
 * FP64 from the cached features (when G/P were current, SVMC_W_DRIFT is set
 * first where G had drifted by more than 1e-8 on its occupied rows). */
svmc_status svmc_refresh(svmc_ctx* ctx, hipStream_t stream);

/* Current configurations.  occ: device int8 (same layout as load); pos
 * (optional): device int16 [W][2][svmc_max_electrons], the site of each
 * electron label (labels start in ascending site order and keep their
 * identity through Metropolis moves), -1 padded. */
svmc_status svmc_get_state(svmc_ctx* ctx, int8_t* occ, int16_t* pos,
                           hipStream_t stream);
int32_t svmc_max_electrons(const svmc_ctx* ctx);

/* d log|psi_w| / d theta (theta layout of svmc_num_params), computed in FP64,
 * for the network of Sec. II.B whose parameters Sec. II.F optimises.
 * vjp_w == NULL: out is device [W][n_params], one row per walker (entries of
 * other lattices' projection and per-site embedding blocks are 0).
 * vjp_w != NULL (device [W]): out is device [n_params] = sum_w vjp_w[w] *
 * d log|psi_w|/d theta, summed in walker order (deterministic).
 * out_prec: element type of out, SVMC_FP64 (double) or SVMC_FP32 (float, each
 * entry rounded once from the FP64 result; halves the Jacobian's memory);
 * other values: SVMC_ERR_INVALID_ARG.
 * Uses d log|det Phi| = tr(Phi^-1 dPhi) for the projection, dH_L = P = W Phi^-1
 * at the occupied sites, and back-propagation through the residual conv stack
 * (pre-activations recomputed from the cached features) to the embedding.
 * Conv weights enter at the values the forward uses; with BF16 conv inputs the
 * activation rounding is not differentiated.  Inverses are rebuilt first if
 * Metropolis moves made them stale.  Walkers flagged SINGULAR, NONFINITE or
 * BADCOUNT get a NaN row and are left out of the VJP sum.  Scratch: up to
 * 4096 walkers x (N C) doubles, plus 1024 x n_params doubles for the VJP or
 * an FP32 Jacobian. */
svmc_status svmc_grad_logpsi(svmc_ctx* ctx, const double* vjp_w, void* out,
                             svmc_prec out_prec, hipStream_t stream);

/* Per-walker flag bits (svmc_walker_flag), device [W] int32. */
svmc_status svmc_walker_flags(svmc_ctx* ctx, int32_t* flags, hipStream_t stream);

/* Symmetry projection (App. B, symmetrized wavefunction):
 *   psi_sym(n) = sum over g of Pi(n, g) chi_g psi(g n).
 * A group element g maps site s to perm[g][s] and, if flip[g], exchanges the
 * two spins; U_g |n> = Pi(n, g) |g n> on Fock states (mapped creation
 * operators put back into the canonical order: spin-up block first,
 * ascending site).  chi: the characters (any finite reals; +-1 for a
 * one-dimensional representation).
 *
 * svmc_set_symmetry: host arrays perm [n_g][N] int32, flip [n_g] int32 (0/1),
 * chi [n_g] FP64, copied.  One-lattice contexts only (UNSUPPORTED
 * otherwise).  INVALID_ARG unless element 0 is the identity, every perm is a
 * permutation, flips have n_up == n_dn, and every element is a symmetry of
 * the Hamiltonian: nearest and next-nearest bonds map to bonds of the same
 * kind and the t-J pinning field is kept.  n_g = 0 removes the group.
 *
 * svmc_sym_expand: device occ [W][N] int8 -> device out [W n_g][N], walker
 * k n_g + g = g n_k.  Load the result with svmc_load_walkers.
 *
 * svmc_local_energy_sym: for a loaded batch of W n_g walkers laid out as
 * svmc_sym_expand writes them, device eloc / sign / logabs [W] and weights
 * [W n_g] (sign, logabs, weights may be NULL): the local energy of psi_sym,
 *   E_sym(n) = sum_g w_g E_loc(g n),  w_g = Pi(n, g) chi_g psi(g n) / psi_sym(n)
 * (the copies' low-rank local energies; exact because every U_g commutes
 * with H), sign and log|psi_sym(n)|, and the copies' weights w_g, so that
 * d log|psi_sym(n)| / d theta = sum_g w_g d log|psi(g n)| / d theta: the
 * gradient is svmc_grad_logpsi with vjp_w[k n_g + g] = c_k w_g for upstream
 * weights c_k.  A walker whose copies are not
 * the images of copy 0 (e.g. after svmc_sweep moved them independently), or
 * with a BADCOUNT copy, gets NaN and SVMC_W_SYMMETRY on copy 0.  psi_sym = 0
 * gives E NaN, sign 0, logabs -inf.  svmc_sweep_sym samples |psi_sym|^2;
 * walkers from svmc_sweep (|psi|^2) serve by reweighting with
 * |psi_sym / psi|^2.  INVALID_ARG if the walker count is not a multiple of
 * n_g; STATE without a group or walkers. */
svmc_status svmc_set_symmetry(svmc_ctx* ctx, int32_t n_g, const int32_t* perm, const int32_t* flip,
                              const double* chi);
svmc_status svmc_sym_expand(svmc_ctx* ctx, int64_t W, const int8_t* occ, int8_t* out, hipStream_t stream);
svmc_status svmc_local_energy_sym(svmc_ctx* ctx, double* eloc, double* sign, double* logabs, double* weights,
                                  hipStream_t stream);

/* Metropolis sampling of |psi_sym|^2 (App. B with Sec. II.A) on a batch laid
 * out as svmc_sym_expand writes it: symmetric walker k draws the proposal
 * of the ordinary sampler (svmc_sweep) from the Philox block with counter
 * (k, step0 + q) and its copy 0's labels; the move is mapped to every copy
 * (site i -> perm[g][i], spin exchanged under flip), each copy's ratio
 * comes from the local update (Sec. II.C), and the move is accepted for all
 * copies iff u < |psi_sym(n') / psi_sym(n)|^2 with
 *   psi_sym(n') / psi_sym(n) = (+-) sum_g a_g R_g / sum_g a_g,  a_g = Pi(n, g) chi_g psi(g n),
 * so the copies stay images of copy 0.  n_accept: device [W n_g] int64 or
 * NULL, incremented per copy.  Errors as svmc_sweep, plus STATE without a
 * group and INVALID_ARG if the walker count is not a multiple of n_g. */
svmc_status svmc_sweep_sym(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed, uint64_t step0, int64_t* n_accept,
                           hipStream_t stream);

/* Launch shape of the low-rank local-energy kernel (not a step of the
 * method; results agree to rounding across shapes):
 *   slices        workgroups each walker's hops are split over (1..64);
 *                 a walker's slices run on one XCD, their partial sums are
 *                 added in slice order;
 *   row_form_max  a hop whose two spins each change at most this many
 *                 orbital rows takes the row form of the determinant lemma,
 *                 det(Phi'[K] Phi^-1[:, K]) of size |K| (padded to 8 or 16),
 *                 otherwise the column form of size C + 1 (Sec. II.C; the two
 *                 are equal by Sylvester's identity): 0 (never), 8 or 16.
 * Defaults: slices 8, row_form_max 16.  svmc_set_launch validates
 * (SVMC_ERR_INVALID_ARG otherwise); svmc_get_launch reports the current one. */
typedef struct {
  int32_t slices, row_form_max;
} svmc_launch;
svmc_status svmc_set_launch(svmc_ctx* ctx, const svmc_launch* launch);
svmc_status svmc_get_launch(const svmc_ctx* ctx, svmc_launch* launch);

/* Autotuner of the low-rank local-energy launch shape (svmc_launch): times
 * svmc_local_energy(LOWRANK) on the loaded walkers for slices in
 * {1, 2, 4, 8, 16, 24, 32} x row_form_max in {0, 8, 16} and keeps, among
 * the shapes within 0.5 % of the fastest, the one with the fewest slices and
 * then the largest row-form limit (so that timing noise does not flip the
 * choice between runs).  cache_path (may be NULL): a text file; a line
 * for the same shape key (lattices, network, precision, walker count,
 * device name) is reused without timing, otherwise the result is appended.
 * *slices_out (may be NULL) receives the chosen slice count.  Synchronises
 * `stream`.  Errors: SVMC_ERR_STATE without walkers. */
svmc_status svmc_tune(svmc_ctx* ctx, const char* cache_path, int32_t* slices_out, hipStream_t stream);

const char* svmc_status_string(svmc_status s);
/* Message of the last error on this context ("" if none). */
const char* svmc_last_error(const svmc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SCALEVMC_H */
