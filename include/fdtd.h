/*
 * fdtd.h -- C ABI of the MI355X (gfx950) imaginary-time FDTD library.
 *
 * Method: Strickland & Yager-Elorriaga, "A Parallel Algorithm for Solving the
 * 3d Schroedinger Equation", arXiv:0904.0939.  A real wavefunction psi on an
 * N^3 lattice of spacing a = L/N (Sec. III) is relaxed in imaginary time by
 * the update of Eq. (updateeq),
 *     psi' = A psi + (B dt / 2m) sum_i (D . Psi-hat)_i,
 *     A = (1 - dt V/2) / (1 + dt V/2),   B = 1 / (1 + dt V/2),
 * with psi = 0 on the ghost sites around the lattice (Sec. III, Sec. V).  Each
 * step also reduces, over the state it reads, the norm, the energy of
 * Eq. (energysum) (taken as +<H>; the printed sign is reversed) and the rms
 * radius, and renormalises the state (Sec. III).
 *
 * Conventions shared by every call:
 *  - Sites i = 0..N-1 per axis sit at x_i = (2i - (N-1)) a/2, centred on the
 *    origin; a field is stored f[(ix*N + iy)*N + iz], z fastest, no padding.
 *  - Every call returns an fdtd_status; no C++ exception crosses the ABI.
 *    fdtd_last_error() gives a thread-local message for the last failure.
 *    A handle stays valid after FDTD_EINVAL and FDTD_ENONFINITE.
 *  - All device work is ordered on the stream given at creation (NULL = the
 *    device's default stream).  Calls that return host values synchronise it.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Host buffers passed in are copied before the call returns and stay owned
 *    by the caller.  Device pointers passed in must stay valid until the call
 *    has completed on the stream.
 *  - The library never falls back to a CPU path: without a usable gfx950 GPU
 *    every call that touches device memory returns FDTD_EHIP.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_ctx* fdtd_t;

typedef enum {
  FDTD_OK = 0,
  FDTD_EINVAL = 1,     /* bad argument; nothing was changed */
  FDTD_ENOMEM = 2,     /* device or host allocation failed, or workspace too small */
  FDTD_EHIP = 3,       /* HIP runtime error (no device, launch failure, ...) */
  FDTD_EUNSTABLE = 4,  /* dt >= m a^2 / 3, the von Neumann bound of Sec. III */
  FDTD_ENOTREADY = 5,  /* call order: potential and initial state must be set first */
  FDTD_ENONFINITE = 6  /* a reduction produced NaN/Inf; the offending step is reported */
} fdtd_status;

/* Storage type of psi (and of user arrays).  V is stored in FP64 when psi is
 * FP64 and in FP32 otherwise.  Arithmetic: FP64 storage computes in FP64;
 * FP32 and BF16 storage compute the update in FP32.  The reductions are
 * always accumulated in FP64. */
typedef enum { FDTD_F64 = 0, FDTD_F32 = 1, FDTD_BF16 = 2 } fdtd_dtype;

/* Analytic potentials, evaluated in FP64 at the site coordinates and rounded
 * to the storage type of V.  p[] holds the parameters listed. */
enum {
  FDTD_POT_CONST = 0,       /* V = p0                                              */
  FDTD_POT_HO = 1,          /* V = (p0^2 x^2 + p1^2 y^2 + p2^2 z^2)/2  (Sec. VII.D)  */
  FDTD_POT_COULOMB = 2,     /* V = -p0 / r                                         */
  FDTD_POT_COULOMB_REG = 3, /* Eq. (coulombpot): 0 for r < a, -p0/r + p0/a else     */
  FDTD_POT_CORNELL = 4,     /* V = -p0/r + p1 r + p2 z^2                           */
  FDTD_POT_WELLS = 5,       /* HO(p0,p1,p2) - sum_k A_k exp(-|r-c_k|^2 / 2 s_k^2);
                               p[3+5k .. 7+5k] = A_k, cx, cy, cz, s_k             */
  FDTD_POT_DODECA = 6       /* Sec. VII.E: V = p0 inside a regular dodecahedron, 0
                               outside; lattice units u = x / ((N-1) a / 2) put
                               the first / last site of each axis at -1 / 1, the
                               vertices at (+-1,+-1,+-1)/phi, (0,+-1/phi^2,+-1)
                               and cyclic (circumradius sqrt(3)/phi); closed,
                               faces with a 1e-12 relative slack               */
};

/* Initial-state kinds (Sec. III: random start; Sec. VI: a coarser solution). */
enum { FDTD_INIT_UNIFORM = 0, FDTD_INIT_GAUSS = 1, FDTD_INIT_USER = 2 };

/* Parity word for the symmetry operators of Sec. IV: two bits per axis
 * (x: bits 0-1, y: bits 2-3, z: bits 4-5); 0 free, 1 S_i, 2 A_i. */
#define FDTD_PARITY(px, py, pz) ((uint32_t)(((px) & 3) | (((py) & 3) << 2) | (((pz) & 3) << 4)))

typedef struct {
  int32_t n;          /* lattice side, 2 <= N <= 8192 (N^3 sites)              */
  int32_t psi_dtype;  /* fdtd_dtype of the stored wavefunction                 */
  double box_len;     /* L = N a > 0                                           */
  double mass;        /* m > 0                                                 */
  double dt;          /* imaginary-time step; must satisfy 0 < dt < m a^2 / 3  */
  double v_inf;       /* V at infinity, for the binding energy (Eq. bindingenergy) */
  int32_t device;     /* HIP device ordinal                                    */
  int32_t history;    /* per-step observable records kept on the device (ring);
                         0 selects 4096                                        */
  void* stream;       /* hipStream_t, or NULL                                  */
} fdtd_config;

/* Observables of one lattice (Sec. III, Eq. energysum, Eq. bindingenergy):
 * norm2 = a^3 sum psi^2 of the stored state, energy = <H>, its kinetic and
 * potential parts, r_rms = sqrt(<r^2>) from the lattice centre,
 * binding = energy - v_inf, tau = step * dt, step = steps taken so far. */
typedef struct {
  double norm2, energy, kinetic, potential, r_rms, binding, tau;
  int64_t step;
} fdtd_obs;

/* Options of fdtd_evolve.
 *  max_steps        steps to run at most (>= 0).
 *  renorm_every     rescale the state to a^3 sum psi^2 = 1 after every k-th
 *                   step (0: never).  The scale is folded into the next
 *                   step's update (exact: the update is linear).
 *  check_every      K > 0: every K steps compare the energy of the state
 *                   entering the K-th step with the previous check and stop
 *                   when |dE| <= rel_tol |E - v_inf| (Sec. V); 0: no check.
 *  reimpose_parity_every  re-apply the set_initial parity every k steps
 *                   (Sec. IV; 0: never -- the update preserves it bit-exactly).
 *  use_graph        1: capture the step loop between two boundaries (check,
 *                   parity, projection; at most 64 steps without a check) in
 *                   a HIP graph, cached per length, and replay it.
 *  project_every    k > 0: after every k-th step, project each member's state
 *                   against its projection states (fdtd_project), so the
 *                   relaxation converges to the lowest state orthogonal to
 *                   them (Sec. III); 0: never.
 *  flags            FDTD_EVOLVE_ASYNC: enqueue the steps on the stream and
 *                   return without waiting for them (check_every must be 0;
 *                   steps_done = max_steps, converged = 0).  A non-finite
 *                   reduction is then reported by the next fdtd_evolve
 *                   without this flag.  For loops that keep the device busy
 *                   and for timing: the calls between two events launch
 *                   only kernels (after the first call of a given length,
 *                   which captures its graphs).  0: wait and check.
 */
#define FDTD_EVOLVE_ASYNC 1
typedef struct {
  int64_t max_steps;
  int32_t renorm_every;
  int32_t check_every;
  int32_t reimpose_parity_every;
  int32_t use_graph;
  double rel_tol;
  int32_t project_every;
  int32_t flags;     /* 0 or FDTD_EVOLVE_ASYNC */
} fdtd_evolve_opts;

/* Counters of a handle since its creation (fdtd_get_counters).
 *  graph_captures  HIP graphs captured by fdtd_evolve (use_graph);
 *  graph_replays   graph launches;
 *  allocations     device and pinned-host allocations the library made for
 *                  the handle (workspace, work items, staging, scratch). */
typedef struct {
  int64_t graph_captures;
  int64_t graph_replays;
  int64_t allocations;
  int64_t reserved;
} fdtd_counters;

/* Launch shape of the fused step kernel (see fdtd_autotune).
 *  vz     sites per lane along z, 1 or the dtype's vector width (F64 2,
 *         F32 4, BF16 8; requires N % vz == 0);
 *  ry     vectors per lane per plane (1, 2 or 4); vz * ry <= 8 (<= 4 for F64);
 *  xchunk at most this many planes streamed per work item: a lattice's N
 *         planes split into ceil(N / xchunk) near-equal x-ranges (>= 1; 0:
 *         the longest stream that still gives every CU a work item); on a
 *         batch, work items run longest first;
 *  grid   work-groups launched (0: one per work item);
 *  xcd_remap  1: order work items so that each XCD's L2 sees neighbouring tiles;
 *  depth  planes of HBM prefetch ahead of the plane being updated (1..3;
 *         1 for vz = 1; 4 and 5 also for two-step passes of F32 and BF16
 *         states, whose odd last step of an evolve then prefetches 3);
 *  variant  0: 256-lane work-groups, y / z neighbours re-read through the
 *         caches, the new state streamed past the caches; 2: the same with
 *         512-lane work-groups (ry = 1); 3: variant 0 storing the new state
 *         written through at system scope, so it stays in the last-level
 *         cache for the next step (vz = the vector width, ry <= 2; the
 *         default for a single lattice whose two state buffers and V fit in
 *         512 MiB); 1: large work-groups (1024 lanes, 512 for BF16) sharing
 *         an LDS copy of each plane (needs vz = the vector width, 2N / vz <=
 *         the work-group size and a tile of at most 64 KiB; ry is ignored);
 *  persist  0: one launch per step (or pass); n > 0: one persistent launch
 *         advances every member up to n steps (variant 0 only), or with
 *         tblock = 2 up to n two-step passes (2n steps, n <= 32768).  Its work-groups (grid,
 *         0: one per CU) take (step, work item) tickets in order; a work item
 *         of step t first waits until its own lattice has finished step t - 1,
 *         so the end of one step overlaps the start of the next on a batch.
 *         Results are bit-identical to per-step launches of the same shape.
 *         A wait is bounded (environment FDTD_PERSIST_SPIN_LIMIT polls,
 *         default 2^22); past it the launch drains and evolve returns
 *         FDTD_EHIP with the state invalid.  Default: 64 for a batch, 0 for
 *         a single lattice;
 *  vfuse  1 (default): on F32 / BF16 lattices whose potentials all came from
 *         fdtd_set_potential_analytic with kinds CONST..CORNELL, the step
 *         evaluates V from the site coordinates in FP32 (hardware 1/sqrt(r^2))
 *         instead of streaming the V table from HBM (12 -> 8 bytes per site for
 *         F32, 8 -> 4 for BF16); variant 0 (per-step or persistent) only, and
 *         not inside fdtd_energy_grad.  V then differs from the table (V computed
 *         in FP64, rounded once) by a few FP32 ulps.  0: always read the table;
 *  tblock  0 (default): one pass over HBM per step; 2: temporal blocking, two
 *         steps per pass (psi and V read once, psi written once per two steps).
 *         Work items are then tiles of the (y, z) plane (F32 and BF16: 32 x
 *         64 sites, or 16 x 128 with tile = 1; F64: 16 x 32) streaming x: a work item first advances its
 *         tile plus a one-site frame around it (and one plane on each side in
 *         x) by one step, in registers and LDS, then its own tile by the
 *         second.  Any lattice side (a multiple of vz), ry = 1, vz = the
 *         vector width, variant 0; persist > 0 runs the passes persistently
 *         (a tile of pass p waits until its lattice has finished pass p - 1;
 *         the same bits as one launch per pass); not inside fdtd_energy_grad.
 *         The rescale can only follow a pass: one due after a pass's first
 *         step (renorm_every) is applied after its second.  With the rescale
 *         off the states are the same bits as one launch per step (shared
 *         per-site arithmetic; BF16: the same rounding bits); the reductions
 *         then differ only in their summation order (per tile instead of per
 *         flattened chunk; BF16 lanes also hold 4 sites instead of 8).  An odd
 *         remainder of steps runs one launch per step;
 *  tile   two-step tile shape of F32 / BF16 states (tblock = 2; 0 otherwise):
 *         0 (default) 32 x 64 sites, 1: 16 x 128.  The wide tile's frame has
 *         half as many column sites (each its own cache line) and more row
 *         sites (contiguous): fewer HBM bytes per pass, more arithmetic for the
 *         frame.  It wins where the pass streams the V table from HBM, and
 *         loses where the pass evaluates V itself or on small lattices; the
 *         same bits either way. */
typedef struct {
  int32_t vz, ry, xchunk, grid, xcd_remap, depth, variant, persist, vfuse, tblock, tile;
} fdtd_tuning;

/* ---- lifetime -------------------------------------------------------------*/

/* Create a handle for one lattice.  Validates the config (FDTD_EINVAL) and the
 * stability bound dt < m a^2/3 (FDTD_EUNSTABLE).  No device memory is taken
 * until fdtd_bind_workspace or the first call that needs it. */
fdtd_status fdtd_create(const fdtd_config* cfg, fdtd_t* out);

/* Create one handle for `count` lattices of possibly different N, box, mass
 * and dt that advance together: one launch per step covers every member.  All
 * members share psi_dtype, device, history and stream (taken from cfgs[0]). */
fdtd_status fdtd_create_batch(const fdtd_config* cfgs, int32_t count, fdtd_t* out);

/* Bytes of device memory the handle needs (fields, reductions, history). */
fdtd_status fdtd_workspace_size(fdtd_t h, size_t* bytes);

/* Use caller-owned device memory (e.g. a torch tensor) of at least
 * fdtd_workspace_size bytes, 256-byte aligned, kept alive until fdtd_destroy.
 * Must precede every other device call; without it the library allocates. */
fdtd_status fdtd_bind_workspace(fdtd_t h, void* dev_ptr, size_t bytes);

/* Release the handle and any memory the library allocated.  NULL is a no-op. */
fdtd_status fdtd_destroy(fdtd_t h);

/* ---- state preparation ----------------------------------------------------*/

/* Set V of `member` from an array of N^3 values (dtype F64 or F32), on the host
 * (on_device = 0) or the device. */
fdtd_status fdtd_set_potential(fdtd_t h, int32_t member, const void* v, int32_t dtype,
                               int32_t on_device);

/* Set V of `member` (-1: every member) from an analytic kind FDTD_POT_*. */
fdtd_status fdtd_set_potential_analytic(fdtd_t h, int32_t member, int32_t kind, const double* p,
                                        int32_t np);

/* Initial state of `member` (-1: every member).  UNIFORM draws U[-1, 1) and
 * GAUSS unit normals (Box-Muller) from counter-based SplitMix64 (Steele, Lea
 * & Flood 2014): draw j of site s of member m is the (2^36 m + 2s + j + 1)-th
 * output of the stream seeded with `seed`.  The parity word then copies the
 * lower half (i < N/2) of each masked axis onto the upper half, with a sign
 * flip for A_i, zeroing the mid plane of odd N under A_i (Sec. IV).  USER
 * copies N^3 values of `dtype` from `user` (host or device) as given: the
 * parity word is then only recorded, for reimpose_parity_every.  Resets the
 * step counter and the history; the state is normalised on entry to the first
 * step (fdtd_checkpoint_load restores a state with its step count). */
fdtd_status fdtd_set_initial(fdtd_t h, int32_t member, int32_t kind, uint64_t seed,
                             uint32_t parity, const void* user, int32_t dtype, int32_t on_device);

/* ---- excited states (Sec. III) ---------------------------------------------*/

/* Keep n states of `member` (n consecutive fields of N^3 values of `dtype`,
 * z fastest, host or device; copied, in the member's arithmetic type) to be
 * projected out by fdtd_project and by evolve's project_every.  n = 0 drops
 * them; at most 16.  Typical use: converged lower states, in order. */
fdtd_status fdtd_set_projection_states(fdtd_t h, int32_t member, const void* states, int32_t n,
                                       int32_t dtype, int32_t on_device);

/* The snapshot method of Sec. III: remove from the current state of `member`
 * its components along the kept states, one after the other in their order,
 *     psi <- psi - phi_k <phi_k|psi> / <phi_k|phi_k>   (sums in FP64),
 * then renormalise.  Applied to a snapshot taken at tau with
 * tau (E_{k+1} - E_k) >> 1 and the k lower states kept, the result estimates
 * the next excited state.  coef (optional, host, n doubles) receives each
 * <phi_k|psi> / <phi_k|phi_k>.  FDTD_EINVAL if no states are kept. */
fdtd_status fdtd_project(fdtd_t h, int32_t member, double* coef);

/* ---- the hot path ----------------------------------------------------------*/

/* Advance every member; see fdtd_evolve_opts.  steps_done and converged
 * (optional) receive the steps run and whether the check was met (for a batch:
 * every member converged).  Returns FDTD_ENONFINITE if a reduction went
 * non-finite; the state is then left as computed. */
fdtd_status fdtd_evolve(fdtd_t h, const fdtd_evolve_opts* opts, int64_t* steps_done,
                        int32_t* converged);

/* Observables of the current state of every member (out[count]): one
 * reduction pass over the lattice(s). */
fdtd_status fdtd_observables(fdtd_t h, fdtd_obs* out);

/* Recorded per-step observables of `member`: for the last `max` steps (at most
 * the history size), out[k] describes the state entering step
 * first_step + k.  count receives the number written. */
fdtd_status fdtd_history(fdtd_t h, int32_t member, fdtd_obs* out, int64_t max, int64_t* count);

/* Copy the state of `member`, normalised to a^3 sum psi^2 = 1, into N^3
 * values of `dtype` (F64, F32 or BF16) at dst (host or device). */
fdtd_status fdtd_get_psi(fdtd_t h, int32_t member, void* dst, int32_t dtype, int32_t on_device);

/* Copy the stored state of `member` exactly as held (its storage dtype, not
 * normalised: the pending renormalisation scale is not applied) to dst (host
 * or device), with the number of steps it has taken.  For bit-level checks
 * and checkpoints; fdtd_set_initial(USER) restores such a copy. */
fdtd_status fdtd_get_state(fdtd_t h, int32_t member, void* dst, int32_t on_device, int64_t* step);

/* Checkpoint and resume.  The paper saves converged wavefunctions and
 * restarts from them (Sec. VII.G); a checkpoint here carries what a
 * relaxation needs to continue exactly where it stopped: a header (magic,
 * version, storage dtype, N, step count, the pending renormalisation scale,
 * the parity word, L and dt) followed by the stored state as held (storage
 * dtype, z fastest).  A run split by save / load takes the same bits as an
 * unsplit one: the step count continues, so tau and the stochastic rounding
 * of BF16 states continue too.
 * size: bytes of a record of `member` (80 + N^3 * element size).
 * save: writes the record to dst (host or device, `size` bytes); synchronises.
 *   FDTD_ENONFINITE if the member's last step went non-finite.
 * load: restores a record into `member` of a handle (the same one or another)
 *   whose member has the same N, dtype, box length and dt (FDTD_EINVAL
 *   otherwise, or for a header that is not a record).  The member's history
 *   ring then starts at the record's step.  src (host or device) is read
 *   before the call returns. */
fdtd_status fdtd_checkpoint_size(fdtd_t h, int32_t member, size_t* bytes);
fdtd_status fdtd_checkpoint_save(fdtd_t h, int32_t member, void* dst, int32_t on_device);
fdtd_status fdtd_checkpoint_load(fdtd_t h, int32_t member, const void* src, int32_t on_device);

/* Multi-resolution reseeding (Sec. VI, Sec. VII.G): trilinear interpolation of
 * the coarse member's state onto the fine member's lattice (same box_len,
 * coarse ghosts zero), normalised; resets the fine member's step counter.  The
 * fine member needs its potential set; psi dtypes may differ. */
fdtd_status fdtd_upsample(fdtd_t coarse, int32_t coarse_member, fdtd_t fine, int32_t fine_member);

/* fdtd_upsample for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, bit for bit, with the kernel's per-work-group partial sums
 * of the norm in a static device array of 1 MiB per GPU (held until the
 * process ends) instead of the fine handle's workspace.  Calls no hipMalloc,
 * hipFree or other allocating routine.  Both handles must already have their
 * device memory (a bound workspace, or any earlier call that set the coarse
 * state and the fine potential): FDTD_ENOTREADY otherwise.  Fine sides above
 * 1620 need more partial sums than the array holds: FDTD_EINVAL.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.  Errors and
 * the remaining behaviour as fdtd_upsample. */
fdtd_status fdtd_upsample_noalloc(fdtd_t coarse, int32_t coarse_member, fdtd_t fine,
                                  int32_t fine_member);

/* Gradient of the energy after `steps` renormalised steps from the current
 * state of a single-lattice handle, held fixed, with respect to V: reverse-mode
 * differentiation of Eq. (updateeq) (adjoint stencil with the same A, B),
 * forward states checkpointed every `checkpoint_every` steps and recomputed
 * segment by segment.  Outputs (each optional):
 *   dE_dV     device FP64 N^3 field dE/dV_i;
 *   dE_dtheta for a potential set by fdtd_set_potential_analytic, with
 *             parameters theta[ntheta] (the ones V was set from: EINVAL
 *             otherwise), the derivatives with respect to theta[wrt[k]] for
 *             k < nwrt <= 64: dE/dtheta_j = sum_i (dE/dV_i) dV_i/dtheta_j with
 *             the analytic dV/dtheta_j of the kind (CONST, COULOMB,
 *             COULOMB_REG, DODECA: j = 0; HO, CORNELL: j < 3; WELLS: every
 *             entry: oscillator frequencies, well amplitudes, centres and
 *             widths);
 *   energy    E after `steps` steps.
 * The handle's state is advanced by `steps` steps, as fdtd_evolve would.
 * Device memory: the workspace bound by fdtd_bind_grad_workspace (FDTD_ENOMEM
 * if it is smaller than fdtd_grad_workspace_size), else a buffer the library
 * allocates on the first call and keeps for later calls (re-allocated only
 * when a call needs more).  On F32 lattices dE/dV accumulates in FP32 within
 * each checkpoint segment and in FP64 across segments. */
fdtd_status fdtd_energy_grad(fdtd_t h, int32_t steps, int32_t checkpoint_every,
                             const double* theta, int32_t ntheta, const int32_t* wrt,
                             int32_t nwrt, void* dE_dV, double* dE_dtheta, double* energy);

/* Device bytes fdtd_energy_grad needs on this single-lattice handle for
 * `steps` steps with checkpoints every `checkpoint_every`: ceil(steps / k)
 * checkpoints and min(k, steps) + 1 recomputed states of N^3 storage values,
 * two adjoint fields, the FP64 dE/dV accumulator (and, on F32 lattices, its
 * FP32 segment accumulator), plus descriptors and 512 KiB of scratch. */
fdtd_status fdtd_grad_workspace_size(fdtd_t h, int32_t steps, int32_t checkpoint_every,
                                     size_t* bytes);

/* Use caller-owned device memory (e.g. a torch tensor; 256-byte aligned, kept
 * alive until fdtd_destroy or the next bind) for fdtd_energy_grad instead of a
 * library allocation; a buffer the library had allocated is freed.  dev_ptr
 * NULL unbinds (later calls allocate again). */
fdtd_status fdtd_bind_grad_workspace(fdtd_t h, void* dev_ptr, size_t bytes);

/* ---- launch shape -----------------------------------------------------------*/

fdtd_status fdtd_get_tuning(fdtd_t h, fdtd_tuning* out);
fdtd_status fdtd_set_tuning(fdtd_t h, const fdtd_tuning* t);

/* Time every valid launch shape of the step kernel on this handle with HIP
 * events, keep the fastest, and cache it per (device architecture and CU
 * count, dtype, lattice sizes, whether the step evaluates V itself) for later
 * handles of this process (and, through
 * fdtd_tune_cache_save / _load, of later processes).  The state, step counters and history
 * are saved first and restored after (the trials step the lattice).  A shape
 * found in the cache is set without timing; best_ms then receives -1.
 * The shapes include two-step passes (tblock = 2), which move a rescale due
 * after a pass's first step to its second (see fdtd_tuning).
 * chosen (optional) receives the shape; best_ms (optional) its time per step. */
fdtd_status fdtd_autotune(fdtd_t h, int32_t steps_per_trial, fdtd_tuning* chosen,
                          double* best_ms);

/* The autotuner's cache as a text file, so that a later process starts from
 * the shapes an earlier one measured.  One line per entry: the key (no
 * spaces; e.g. gfx950/256cu:1:512 for one F32 lattice of side 512 whose step
 * reads the V table, gfx950/256cu:1:512:fv when it evaluates V itself), then the
 * eleven fdtd_tuning fields in their declaration order; lines starting with '#'
 * are comments.
 * save: writes every entry of this process's cache to `path` (created or
 *   truncated).  EINVAL if the file cannot be written.
 * load: replaces this process's cache with the entries of `path`.  EINVAL
 *   (cache unchanged) if the file cannot be read or a line is malformed.  An
 *   entry is checked only when fdtd_autotune finds it: one the handle rejects
 *   (fdtd_set_tuning fails) is dropped and the shapes are timed anew.
 * Neither touches the GPU; both are thread-safe. */
fdtd_status fdtd_tune_cache_save(const char* path);
fdtd_status fdtd_tune_cache_load(const char* path);

/* ---- misc -------------------------------------------------------------------*/

/* Wait for all work of the handle. */
fdtd_status fdtd_synchronize(fdtd_t h);

/* The handle's counters (see fdtd_counters); no device work. */
fdtd_status fdtd_get_counters(fdtd_t h, fdtd_counters* out);

/* Number of members, and the stream the handle launches on. */
fdtd_status fdtd_info(fdtd_t h, int32_t* count, void** stream);

const char* fdtd_status_string(fdtd_status s);
const char* fdtd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_H */
