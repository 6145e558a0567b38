/*
 * fmm_mc.h -- C ABI of the MI355X (gfx950) library for Metropolis-Hastings
 * Monte Carlo of point charges in a periodic cube with the multilevel
 * local-expansion method of Saunders, Grant & Mueller (arXiv:2006.16622).
 *
 * Physics and units. N point charges q_i at positions r_i in the periodic
 * cube [0, box)^3, Gaussian units (k_e = 1): the energy is
 *   U = 1/2 sum_{i,j} sum'_{nu in Z^3} q_i q_j / |r_i - r_j + box nu|
 * with tin-foil (conducting) boundary conditions at infinity. The charges
 * must sum to zero.
 *
 * The method (Sec. 3.2 of the paper): an octree of L = levels + 1 levels,
 * level l having 8^(l-1) cells (Sec. 3.1); each cell of every level l >= 2
 * keeps a degree-p local expansion Psi^Delta of the charges in its
 * interaction list only (Eq. DeltaPsiSum, Eq. local_expansion); images of
 * the 27-box extended domain take part (Sec. 3.4), the rest of the periodic
 * lattice enters through the moments K, E and the lattice operator R
 * (Sec. 3.4). A proposal costs O(p^2 L) (Alg. L.1 + Alg. 1), an accepted
 * move O(189 p^2 L) (Alg. L.2).
 *
 * Memory. The caller allocates one device workspace per chain (size from
 * fmm_mc_workspace_bytes) and owns it; the library never frees it. Host
 * arrays passed in are copied; the caller keeps ownership. Constant tables
 * (translation operators, lattice operator) are shared by every chain of
 * the same degree on a device and are allocated by the library on first
 * use; fmm_mc_release_tables() frees them.
 *
 * Streams. Every call enqueues on the HIP stream given at setup and waits
 * for it before returning a host value. Handles are not thread-safe;
 * distinct handles are independent.
 *
 * Errors. Every entry point returns FMM_MC_OK (0) or a negative code below;
 * no exception or exit crosses the ABI. fmm_mc_strerror() names a code.
 */
#ifndef FMM_MC_H
#define FMM_MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_MC_OK 0
#define FMM_MC_EINVAL (-1)      /* bad argument (p, levels, box, n, null pointer) */
#define FMM_MC_ERANGE (-2)      /* particle index out of range */
#define FMM_MC_ENONNEUTRAL (-3) /* |sum q| > 1e-12 sum |q| */
#define FMM_MC_ESINGULAR (-4)   /* new position coincides with another charge */
#define FMM_MC_ENOMEM (-5)      /* workspace too small */
#define FMM_MC_EDEVICE (-6)     /* a HIP call failed */
#define FMM_MC_EOVERFLOW (-7)   /* a leaf cell exceeded its capacity */
#define FMM_MC_ESTATE (-8)      /* handle not set up / inconsistent chains */

/* flags */
#define FMM_MC_MIXED 0x1u /* FP32 L2P, near field and setup M2L; FP64 elsewhere */
/* The multipole-based variant of Sec. 3.3 (Alg. M.1-M.3) in place of the
 * local-expansion method: each level keeps the multipole expansion of every
 * cell; a proposal evaluates the multipoles of the interaction lists of the
 * old and new cell on every level at the charge (2 x 189 x (L-1) M2P), an
 * accept updates one multipole per level and side. Near field, self-image,
 * far-lattice and tin-foil terms are those of the local method. The setup
 * forms the multipoles by P2M and M2M (the result of Alg. M.3 up to
 * rounding) and no local expansions; fmm_mc_dump_locals then returns
 * FMM_MC_ESTATE. FP64 only: combined with FMM_MC_MIXED it is rejected with
 * FMM_MC_EINVAL. Chains of one fmm_mc_run must all use the same variant. */
#define FMM_MC_MULTIPOLE 0x2u
/* Initialise the local expansions by direct P2L, Alg. L.3 (the paper's own
 * initialisation, Sec. 3.2): every charge is added to the expansion of
 * every cell in the interaction list of its cell on every level, images
 * included, in place of the M2L pass. Always FP64; it also serves the
 * re-setup. O(189 p^2 N L) work; the workspace holds extra chunk rows for
 * it (fmm_mc_workspace_bytes with this flag). Not with FMM_MC_MULTIPOLE
 * (FMM_MC_EINVAL). */
#define FMM_MC_DIRECT_SETUP 0x4u
/* Free-space boundary conditions (Sec. 3.4): the box [0, box)^3 is the whole
 * domain. No periodic images: interaction lists and near regions keep only
 * cells inside the box (the lists of levels 1 and 2 are empty), the self
 * correction keeps only the charge's own old position, and there is no
 * far-lattice or tin-foil term. Positions are not wrapped: every initial
 * position must lie inside the box (else FMM_MC_EINVAL), a proposal out of
 * the box has dE = +inf (it is never accepted by fmm_mc_run), and
 * fmm_mc_accept of such a move returns FMM_MC_EINVAL. Combines with every
 * other flag. */
#define FMM_MC_FREE_SPACE 0x8u

typedef struct fmm_mc_ctx *fmm_mc_t;

/* Device workspace (bytes) one chain needs: n charges, octree depth
 * `levels` (8^levels leaf cells, so L = levels + 1 levels), degree p.
 * levels in [1, 7], p in [0, 24], n >= 2. */
int fmm_mc_workspace_bytes(int64_t n, int levels, int p, uint32_t flags, size_t *bytes);

/* Initialise a chain: copy pos (n x 3, AoS, host) and q (n, host), wrap the
 * positions into [0, box)^3 (x - box floor(x/box); a result equal to box
 * becomes 0), bin them into the leaf cells, and build every local expansion
 * by the FMM passes P2M -> M2M -> M2L over each interaction list on levels
 * 2..L (the initialisation variant of Sec. 3.2 with no L2L), plus the
 * periodic moments K, E, the lattice term H = R(K) and the dipole (Sec.
 * 3.4). dev_ws: device pointer to at least ws_bytes bytes (from
 * fmm_mc_workspace_bytes), 256-byte aligned, owned by the caller and kept
 * alive until fmm_mc_destroy. hip_stream: a hipStream_t (NULL = default).
 * On success *out receives the handle. */
int fmm_mc_setup(fmm_mc_t *out, void *dev_ws, size_t ws_bytes, void *hip_stream, int64_t n,
                 const double *pos, const double *q, double box, int levels, int p,
                 uint32_t flags);

/* Set up n_chains chains of the same degree p in one pass (the batched
 * form of fmm_mc_setup, for the batched chain loop of fmm_mc_run): every
 * setup kernel runs once over all chains, and the M2L of every level of
 * every chain is one launch, because the scaled translation operators do
 * not depend on the level (Sec. 3.2 initialisation, Sec. 3.4 lattice).
 * Arrays of length n_chains: dev_ws (device workspaces, each 256-byte
 * aligned and at least ws_bytes[c] = fmm_mc_workspace_bytes(n[c],
 * levels[c], p, flags) bytes, owned by the caller), n, pos (host n[c] x 3
 * AoS), q (host n[c]), box, levels. All chains use hip_stream and the
 * current device. On success out[c] receives chain c's handle; on failure
 * no handle is left open and the first error is returned. The library
 * holds two small stream-ordered device allocations (chain descriptors and
 * the M2L tile list) for the duration of the call. */
int fmm_mc_setup_batch(fmm_mc_t *out, int n_chains, void *const *dev_ws, const size_t *ws_bytes,
                       void *hip_stream, const int64_t *n, const double *const *pos, const double *const *q,
                       const double *box, const int *levels, int p, uint32_t flags);

/* Energy change of moving charge idx to new_pos (3 doubles, host, absolute;
 * wrapped by the library): Alg. L.1 plus Alg. 1 with the periodic
 * modifications of Sec. 3.4 (self-image correction, far lattice, tin-foil
 * dipole term). Pure: the state does not change. *dE (host) receives the
 * energy difference. */
int fmm_mc_propose(fmm_mc_t h, int64_t idx, const double *new_pos, double *dE);

/* Accept the move of charge idx to new_pos: Alg. L.2 over every level with
 * images (Sec. 3.4), the K/E/dipole update, the position and the leaf bins.
 * If dE_in is NULL the move is proposed first (the library tracks the total
 * energy, Sec. 4.1); otherwise *dE_in is taken as the energy change. If
 * dE_out is non-NULL it receives the energy change used. */
int fmm_mc_accept(fmm_mc_t h, int64_t idx, const double *new_pos, const double *dE_in,
                  double *dE_out);

/* Options of the on-device Metropolis-Hastings loop. */
typedef struct {
  double beta;      /* inverse temperature in units of a / q^2 */
  double max_step;  /* displacement half-width per component (0 = per-chain value below) */
  const double *chain_max_step; /* host array of n_chains half-widths, or NULL */
  int64_t t0;       /* first step index of the Philox counter */
  int32_t mode;     /* 0 = automatic, 1 = one workgroup per chain, 2 = whole GPU per chain */
  int32_t resetup_every; /* > 0: after this many accepted moves a chain's expansions are rebuilt
                          * from its positions in FP64 (fmm_mc_resetup) before it continues;
                          * 0 = never. Bounds the drift of the accumulated updates. */
  /* optional traces (device pointers, NULL = off), indexed [chain * steps + t] */
  int64_t *trace_idx;
  double *trace_newpos; /* 3 per step */
  double *trace_dE;
  uint8_t *trace_acc;
} fmm_mc_run_opts;

typedef struct {
  int64_t proposed, accepted, singular;
  double dE_sum;    /* sum of accepted dE */
  double energy;    /* running total energy after the run */
  int32_t status;   /* FMM_MC_OK or an error code raised on the device */
  int32_t pad;
  /* device time of the chain's proposing workgroup, microseconds (100 MHz
   * realtime counter): proposals (without the waits), its own share of
   * accepted-move updates, and waiting for the other workgroups' shares
   * (whole-GPU mode only; after an accept that wait comes inside the next
   * proposal, just before it reads the local expansions) */
  double t_propose_us, t_accept_us, t_wait_us;
} fmm_mc_stats;

/* Run `steps` Metropolis-Hastings steps on each chain, on the device. Step t
 * of chain c draws from Philox4x64-10 with key (seed, c) and counter
 * (t0 + t, 0, 0, 0): idx = floor(w0 N / 2^64), displacement component k =
 * max_step (2 ((w_k >> 11) 2^-53) - 1); counter (t0 + t, 1, 0, 0) gives
 * u = (w0 >> 11) 2^-53. The move is accepted iff u < exp(-beta dE)
 * (Sec. 4.1, Sec. 5.1: P = exp(-dU / kT)); a singular move is rejected.
 * All chains must live on the same device and stream. stats (host, n_chains
 * entries) receives per-chain counters. */
int fmm_mc_run(fmm_mc_t *chains, int n_chains, int64_t steps, uint64_t seed,
               const fmm_mc_run_opts *opts, fmm_mc_stats *stats);

/* Most chains one fmm_mc_run_noalloc call takes. */
#define FMM_MC_NOALLOC_MAX_CHAINS 1024

/* fmm_mc_run for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation. Same
 * arguments, semantics and results as fmm_mc_run, bit for bit. It calls no
 * hipMalloc, hipFree or other allocating routine: the launch arguments and
 * per-chain results of a run of several chains (which fmm_mc_run keeps in
 * buffers it allocates on first use) live in a fixed device array of 1 MiB
 * that each GPU the library runs on holds until the process ends, and in a
 * host staging block allocated once by the first fmm_mc_setup of the
 * process; a run of one chain on the whole GPU uses only its workspace, as
 * in fmm_mc_run. Limits: n_chains <= FMM_MC_NOALLOC_MAX_CHAINS (more:
 * FMM_MC_ENOMEM, before anything is touched); opts->resetup_every must be 0
 * (a re-setup builds its graph on first use; FMM_MC_EINVAL otherwise).
 * Every call on one GPU shares that GPU's array (every call writes all of
 * the part it reads): calls that overlap on one GPU race, and calls from
 * several host threads are serialised by a lock. */
int fmm_mc_run_noalloc(fmm_mc_t *chains, int n_chains, int64_t steps, uint64_t seed,
                       const fmm_mc_run_opts *opts, fmm_mc_stats *stats);

/* Fixed-list mode: m proposals (idx[m], new_pos[m x 3], uniforms u[m], all
 * host) applied in order with the rule u < exp(-beta dE). Outputs (host,
 * may be NULL): dE[m], acc[m] (0/1), leaf[m] = leaf cell of the wrapped
 * new position (x + n (y + n z) with n = 2^levels). */
int fmm_mc_replay(fmm_mc_t h, int64_t m, const int64_t *idx, const double *new_pos,
                  const double *u, double beta, double *dE, uint8_t *acc, int32_t *leaf);

/* Total energy of the current state (Sec. 3.2, 3.4), summed on the device. */
int fmm_mc_energy(fmm_mc_t h, double *U);

/* Running energy: energy at setup plus every accepted dE. */
int fmm_mc_running_energy(fmm_mc_t h, double *U);

/* Current (wrapped) positions, n x 3 host array. */
int fmm_mc_get_positions(fmm_mc_t h, double *pos);

/* Local expansion coefficients of every cell on `level` (2..L), written to
 * host out[cell * (p+1)^2 + n*n + n + m]: for m >= 0 the real part of
 * L_n^m, for m < 0 the imaginary part of L_n^{|m|}, in the paper's
 * normalisation (Psi = sum L_n^m rho^n Y_n^m with Y_n^m =
 * sqrt((n-|m|)!/(n+|m|)!) P_n^|m| e^{i m phi}, no Condon-Shortley phase);
 * cells ordered x + n (y + n z). */
int fmm_mc_dump_locals(fmm_mc_t h, int level, double *out);

/* Multipole expansion coefficients of every cell on `level` (1..L), in the
 * layout of fmm_mc_dump_locals: M_n^m = sum q rho^n Y_n^{-m} about the cell
 * centre, Eq. (multipole_expansion_coefficients). For the multipole-based
 * variant this is its live state; for the local method, the multipoles of
 * the last setup. */
int fmm_mc_dump_multipoles(fmm_mc_t h, int level, double *out);

/* Rebuild every expansion from the current (device-resident) positions:
 * the whole setup pass of fmm_mc_setup, captured into a HIP graph on the
 * first call (on a private non-blocking stream) and replayed on the
 * handle's stream afterwards. The running energy is replaced by the fresh
 * total energy; the setup energy is kept. A bin overflow is reported as
 * FMM_MC_EOVERFLOW. */
int fmm_mc_resetup(fmm_mc_t h);

/* Volume move, a move type beyond the single-charge displacement (the
 * paper's outlook, Sec. 6): every position is scaled about the origin by
 * s = new_box / box and the box side becomes new_box. The chain is first
 * re-set up in FP64 from its current positions (as fmm_mc_resetup), then set
 * up again from the same positions scaled by s in the new box; *dE (host)
 * receives the difference of the two setup energies, U(scaled) - U(current).
 * The scaled state becomes the chain's state (running and setup energy
 * U(scaled)). The acceptance rule of the ensemble (for example
 * exp(-beta (dE + P dV)) (V'/V)^N at constant pressure) belongs to the
 * caller, as the Metropolis loop does (Sec. 4.1); to reject, call
 * fmm_mc_rescale_undo. Free space: positions scale about the corner of the
 * box at the origin, and stay inside it. Errors: FMM_MC_EINVAL for a box
 * that is not finite and positive, FMM_MC_EOVERFLOW if a leaf bin overflows
 * (the state is then the last one set up). */
int fmm_mc_rescale(fmm_mc_t h, double new_box, double *dE);

/* Undo the last fmm_mc_rescale of this chain: the box side and every
 * position return to their values before it, bit for bit, and the
 * expansions are set up afresh (FP64) from them. Valid only right after
 * fmm_mc_rescale, before any other call that changes the chain (a run,
 * an accept, a re-setup); FMM_MC_ESTATE otherwise. */
int fmm_mc_rescale_undo(fmm_mc_t h);

/* Result of fmm_mc_autotune. */
typedef struct {
  int32_t m2l_rows;              /* chosen M2L output rows per workgroup: 96 or 192 */
  int32_t helpers;               /* chosen helper workgroups of the whole-GPU run */
  int32_t n_helper_candidates;
  int32_t pad;
  double m2l_ms[2];              /* M2L time (ms) with 96 and with 192 rows per workgroup */
  int32_t helper_candidates[8];
  double step_us[8];             /* time per MH step (us) of each helper candidate */
} fmm_mc_tuning;

/* Autotune the launch shapes for this chain's shape: the M2L output tile
 * (96 or 192 coefficient rows per workgroup; both give identical results)
 * is timed on the chain's data, and the number of helper workgroups of the
 * whole-GPU run (mode 2) is timed over `steps` MH steps (0 = 1000) with
 * inverse temperature beta and displacement half-width max_step, each
 * candidate from the same clone of the chain's state, twice (the faster
 * time counts); fewer helpers than accept blocks are chosen only when more
 * than 2 % faster. Untuned shapes use 96 rows and one helper per block. The chain itself is
 * not changed: the library allocates a temporary copy of the workspace for
 * the trials and frees it before returning. The fastest choices apply to
 * this handle and to every later fmm_mc_setup / fmm_mc_setup_batch of the
 * same device, degree, depth and precision in this process. out (may be
 * NULL) receives the measurements. */
int fmm_mc_autotune(fmm_mc_t h, int64_t steps, double beta, double max_step, fmm_mc_tuning *out);

/* Set the number of helper workgroups of this chain's whole-GPU runs (mode
 * 2), the choice the autotuner makes: 0 = one helper per accept block (the
 * untuned default); a smaller count gives each helper several blocks, and a
 * run raises it as far as needed for the busiest helper's blocks to fit its
 * LDS. Applies to this handle only. Returns FMM_MC_EINVAL for a null handle
 * or a negative count. */
int fmm_mc_set_helpers(fmm_mc_t h, int helpers);

/* Release the handle (not the caller's workspace). */
int fmm_mc_destroy(fmm_mc_t h);

/* Free the shared constant tables of the current device. */
int fmm_mc_release_tables(void);

/* Timing of the device kernels of the last call on this handle, in ms,
 * measured with HIP events on the handle's stream: out[0] = whole call,
 * out[1] = setup M2L (setup only). */
int fmm_mc_last_timing(fmm_mc_t h, double *out, int nout);

const char *fmm_mc_strerror(int code);

/* Host-only diagnostic (no device needed): the constant operators exactly as
 * the library builds them for degree p, in the real coefficient layout of
 * fmm_mc_dump_locals, on cell-size-scaled coefficients (multipoles divided by
 * h^n, locals multiplied by h^(n+1)). kind 0: M2L operator for interaction-
 * list offset o[0..2] (source cell minus target cell, in cells; Sec. 3.1),
 * element out[in * (p+1)^2 + out]; kind 1: M2M operator of the child octant
 * o[0] (bit k = upper half along axis k), same element order; kind 2: the
 * periodic lattice operator R of Sec. 3.4 (box-scaled), element
 * out[out * (p+1)^2 + in]. out: (p+1)^4 doubles, host, caller-owned. */
int fmm_mc_host_operator(int kind, int p, const int *o, double *out);

#ifdef __cplusplus
}
#endif
#endif /* FMM_MC_H */
