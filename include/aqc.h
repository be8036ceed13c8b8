/*
 * aqc.h -- C ABI of the MI355X engine for the time-dependent Schroedinger
 * equation with Hamiltonians in compact Pauli-string ("SQH") form.
 *
 * Method: M. Hofmann, G. Schaller, "Probing nonlinear adiabatic paths with a
 * universal integrator", arXiv:1311.3938.
 *   - state and basis:   Sec. II.A, eq. (ztensor), eq. (expansion)
 *   - Hamiltonian form:  Sec. II.A, eq. (SQH-Hamiltonian), time-dependent
 *                        coefficients m_l(t) at the end of Sec. II.A
 *   - paths:             Sec. II.B eq. (aqc); Sec. IV.A eq. (nlpath)
 *   - time stepping:     Sec. II.B eq. (schroedinger), the 4th-order
 *                        predictor-corrector with one H|psi> per step
 *   - success measures:  Sec. III.B (P_1(T) = |<psi(T)|w>|^2, energy E(T))
 *
 * Conventions shared by every entry point
 *   - qubit q (1-based) is bit q-1 of the basis index z (eq. (ztensor));
 *     |0>, |1> are the sigma^z eigenvectors (+1, -1).
 *   - a state of n qubits is 2^n complex amplitudes, interleaved (re, im),
 *     contiguous, in device memory: AQC_C64 = 2 x float32 (8 bytes),
 *     AQC_C128 = 2 x float64 (16 bytes).  Pointers must be 16-byte aligned.
 *     The caller owns every state and workspace buffer; the library never
 *     allocates state-sized memory.
 *   - a Pauli string is two masks: bit q-1 of x set <=> sigma^x or sigma^y on
 *     qubit q; bit q-1 of z set <=> sigma^z or sigma^y on qubit q (sigma^y sets
 *     both).  sigma^y = [[0,-i],[i,0]].
 *   - hbar = 1; times and energies share one unit.
 *   - every call returns an aqc_status; on failure aqc_last_error() gives a
 *     message (per calling thread).  No call throws across the ABI.  All
 *     device work is enqueued on the context's stream; calls that return host
 *     scalars (reductions, evolve statistics) synchronise that stream.
 *   - floating point: AQC_C64 keeps states in complex64 and forms H|psi> and
 *     the stage updates in float32; every norm, overlap, energy, error
 *     estimate, step-size decision and phase is computed in float64.  AQC_C128
 *     is float64 throughout.
 */
#ifndef AQC_H
#define AQC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int aqc_status;
#define AQC_OK         0
#define AQC_EINVAL    -1  /* bad argument (null pointer, size, mask, value)   */
#define AQC_ENOMEM    -2  /* caller-provided workspace too small               */
#define AQC_EDEVICE   -3  /* HIP runtime error                                 */
#define AQC_EUNSTABLE -4  /* norm guard tripped, or step above stability limit */
#define AQC_ENOTSUP   -5  /* unsupported size or dtype (n > 34)                */
#define AQC_EBUSY     -6  /* no free slot or memory in a batch                 */

typedef enum { AQC_C64 = 0, AQC_C128 = 1 } aqc_dtype;

/* ---- schedules and paths (time dependence of the coefficients) --------- */
typedef enum {
  AQC_SCHED_CONST  = 0,  /* f = 1                                            */
  AQC_SCHED_POLY_S = 1,  /* f = sum_{d<=degree} coef[d] s^d on s_lo <= s < s_hi
                            (s <= s_hi when hi_closed), 0 outside             */
  AQC_SCHED_TRIG_T = 2,  /* f = amp * cos(omega t + phase)                   */
  AQC_SCHED_PWL_S  = 3   /* piecewise linear in s through the knots
                            (s_i, v_i) = (coef[2i], coef[2i+1]), i = 0..degree
                            (degree 0..3, s_i nondecreasing): f = v_0 for
                            s < s_0, v_degree for s >= s_degree, linear in
                            between; at a repeated knot the later value holds.
                            One such ramp per clause expresses the
                            clause-by-clause path, eq. (cbc)-(kpath).         */
} aqc_sched_kind;

typedef struct {
  int32_t kind;       /* aqc_sched_kind                                      */
  int32_t degree;     /* POLY_S: 0..7; PWL_S: knots - 1, 0..3                 */
  int32_t hi_closed;  /* POLY_S: 1 => the window includes s_hi               */
  int32_t reserved;
  double coef[8];
  double s_lo, s_hi;  /* POLY_S window (use +-INFINITY for none)             */
  double amp, omega, phase;
} aqc_sched;

typedef enum {
  AQC_PATH_LINEAR = 0,  /* s(t) = t / T                 (eq. (aqc))          */
  AQC_PATH_SIN2   = 1   /* s(t) = sin^2(pi t / (2 T))                        */
} aqc_path_kind;

typedef struct {
  int32_t kind;
  int32_t reserved;
  double T;
} aqc_path;

typedef struct aqc_ctx aqc_ctx;
typedef struct aqc_ham aqc_ham;

/* ---- context ------------------------------------------------------------ */
/* Binds a device and a HIP stream (hipStream_t passed as void*, NULL = the
 * default stream).  The stream is borrowed, never destroyed.  The context owns
 * small device buffers for reduction partials (a few MB).
 * aqc_destroy waits for the stream and releases the caller's hold on the
 * context; each batch created on it holds it too, so its memory goes with
 * the last of them, and batches and their context may be destroyed in either
 * order (e.g. by finalizers).  A batch whose context was destroyed refuses
 * admit, step, poll and retire (AQC_EINVAL) and can only be destroyed.
 * Destroying a context twice is AQC_EINVAL while a batch still holds it, and
 * undefined after that.                                                      */
aqc_status aqc_create(int device, void* stream, aqc_ctx** out);
aqc_status aqc_destroy(aqc_ctx* ctx);
/* aqc_set_stream waits for the context's current stream before switching.  */
aqc_status aqc_set_stream(aqc_ctx* ctx, void* stream);
/* aqc_trim: the device buffers of released Hamiltonian tables (aqc_ham_free,
 * a replaced plan) are kept and reused by later Hamiltonians once every
 * stream the library launches on has passed the release, because freeing
 * device memory waits for every stream of the device; up to 1 GiB per device
 * is kept.  aqc_trim waits for those releases and frees the kept buffers of
 * `device`.  AQC_EINVAL for a device index outside 0..63.                   */
aqc_status aqc_trim(int device);
const char* aqc_last_error(void);
const char* aqc_version(void);

/* ---- Hamiltonian -------------------------------------------------------- */
/* aqc_build_hamiltonian: H(t) = sum_l weight[l] * f_{sched_id[l]}(t) * P_l
 * (eq. (SQH-Hamiltonian) with time-dependent coefficients), P_l the Pauli
 * string (x_mask[l], z_mask[l]).  Inputs are host arrays of n_terms entries and
 * are copied; the caller keeps ownership.  Terms with equal (x, z, sched_id)
 * are merged; terms with x = 0 form the diagonal, the others are grouped by
 * their flip pattern x.  Errors: EINVAL for n_qubits < 1, masks >= 2^n,
 * non-finite weights, a sched_id outside [0, n_sched), n_sched > 32, bad
 * schedule or path data; ENOTSUP for n_qubits > 34.  The compiled tables live
 * in library-owned device memory (small: O(terms + 2^(n-13) n) entries) until
 * aqc_ham_free.  Up to 26 qubits the tables of both dtypes are built here;
 * larger Hamiltonians build them at their first use.  The context's stream
 * is used for uploads.                                                      */
aqc_status aqc_build_hamiltonian(aqc_ctx* ctx, int n_qubits, int64_t n_terms,
                                 const uint64_t* x_mask, const uint64_t* z_mask,
                                 const double* weight, const int32_t* sched_id,
                                 int n_sched, const aqc_sched* scheds,
                                 const aqc_path* path, aqc_ham** out);
/* aqc_ham_free returns without waiting for the device: launches already
 * queued may still read the tables, whose buffers go to the pool that
 * aqc_trim describes.  NULL is a no-op.                                     */
aqc_status aqc_ham_free(aqc_ham* ham);

typedef struct {
  int32_t n_qubits;
  int32_t n_terms;        /* after merging                                    */
  int32_t n_diag_terms;
  int32_t n_groups;       /* distinct flip patterns x != 0                    */
  int32_t n_passes[2];    /* tile passes per H|psi>, [C64, C128]              */
  int32_t tile_bits[2];   /* bits held on chip by the last pass, [C64, C128]  */
  double spec_lo, spec_hi;/* spectral enclosure of H(t) over [0, T]          */
} aqc_ham_info_t;
aqc_status aqc_ham_info(const aqc_ham* ham, aqc_ham_info_t* out);

/* Tiling of the tile passes for this Hamiltonian and dtype (replaces the
 * default and rebuilds the plan: here up to 26 qubits, else at the next use;
 * synchronises the device).
 * tbf: bits of the last pass's contiguous tile (1..14 complex64, 1..13
 * complex128); tbh: bits of a high-pass tile; lh: its contiguous low bits
 * (1 <= lh < tbh).  options, bits 0-1: how single-qubit flips above the last
 * tile run: 0 in tile passes, 1 in register hypercube passes of the width the
 * library picks for n, 2 in narrow register passes (one wave per hypercube),
 * 3 in wide ones (eight waves of a workgroup span three more bits and trade
 * vertices through LDS); bit 2 (value 4): the other flip patterns above the
 * tile are applied by the last pass, which reads their partners from the
 * source vector (stream groups), instead of by tile high passes.  Stream
 * groups add one vector to the evolve workspace (a second y^p buffer), so
 * query the workspace size after this call.  EINVAL for values out of range,
 * ENOTSUP when some flip pattern does not fit the tiles (the old tiling stays).
 * Used by the autotuner.                                                     */
aqc_status aqc_ham_set_tiling(aqc_ham* ham, int dtype, int tbf, int tbh, int lh,
                              int options);

/* Spectral enclosure [lo, hi] of H(t) on [t0, t1]: exact minimum and maximum of
 * each schedule's diagonal part (device reduction) combined with the triangle
 * inequality for the flip terms, over a grid of 257 times (Weyl bound).      */
aqc_status aqc_spectral_bounds(aqc_ctx* ctx, const aqc_ham* ham, double t0, double t1,
                               double* lo, double* hi);

/* ---- H|psi> ------------------------------------------------------------ */
/* psi_out = H(t) psi_in (the matrix-free product of Sec. II.A).  Device
 * pointers to 2^n amplitudes of `dtype`; psi_in != psi_out (EINVAL).  When the
 * Hamiltonian needs more than one tile pass, `workspace` must hold one state
 * vector (aqc_apply_workspace_bytes); otherwise it may be NULL.             */
size_t aqc_apply_workspace_bytes(const aqc_ham* ham, int dtype);
aqc_status aqc_apply(aqc_ctx* ctx, const aqc_ham* ham, double t, const void* psi_in,
                     void* psi_out, int dtype, void* workspace, size_t ws_bytes);

/* ---- time evolution ----------------------------------------------------- */
#define AQC_METHOD_PC4 0   /* one-evaluation 4th-order predictor-corrector   */
#define AQC_METHOD_RK4 1   /* classical 4-stage Runge-Kutta                  */

#define AQC_SHIFT_VALUE  0 /* subtract opts.shift from H                     */
#define AQC_SHIFT_CENTER 1 /* subtract the midpoint of the spectral enclosure */

/* A chain of fixed-step pc4 calls (aqc_evolve_opts.carry).  The multistep
 * method needs the history of its last steps (Sec. II.B); a call that starts
 * from a plain state rebuilds it with three RK4 steps.  With a carry, each call
 * of a chain continues the previous call's grid and history instead, so a
 * long evolution done in pieces performs exactly the steps of one call.
 * Fill valid = 0 to start a chain; the call fills the rest.  A call with
 * valid = 1 must use the same Hamiltonian, dtype, psi and workspace (whose
 * history vectors the caller leaves untouched), t0 = the previous t1 and the
 * same step; it keeps the chain's shift whatever opts.shift_mode says.
 * Within a chain psi is left in the frame of the shifted Hamiltonian: after a
 * call, psi(t1) = phase * psi (phase_re + i phase_im), a unit factor the
 * caller applies when it needs the state itself (|psi|^2 and the fidelity of
 * Sec. III.B do not depend on it).  EINVAL when a continued call does not
 * match its chain.                                                           */
typedef struct {
  int32_t valid;        /* 0: start a chain; 1: continue it                   */
  int32_t sub;          /* internal position in the step                      */
  int32_t ypc;          /* internal: current y^p buffer                       */
  int32_t dtype;
  int64_t k;            /* steps taken since t_start                          */
  double t_start;       /* grid of the chain: t_start + k h                   */
  double h;
  double shift;         /* the chain's shift                                  */
  double t_ref;         /* frame reference: psi = exp(i shift (t - t_ref)) psi(t) */
  const void* ham;
  const void* psi;
  const void* workspace;
  double phase_re, phase_im;  /* out: psi(t1) = phase * psi                  */
} aqc_pc4_carry;

typedef struct {
  int32_t method;       /* AQC_METHOD_*                                       */
  int32_t n_steps;      /* > 0: fixed steps h = (t1-t0)/n_steps; 0: adaptive  */
  int32_t shift_mode;   /* AQC_SHIFT_*                                        */
  int32_t check_every;  /* norm guard period in steps (0 = off)              */
  double shift;         /* used with AQC_SHIFT_VALUE                          */
  double norm_tol;      /* guard: | ||psi||^2 - ||psi0||^2 | <= norm_tol      */
  double stab_limit;    /* pc4: refuse h*rho above this (<= 0: no check)     */
  /* adaptive pc4 (n_steps == 0): Milne estimate per step, windows of
   * `window` steps, reject above atol (h/2), grow below atol/64 (2h)         */
  double atol, h0, hmin, hmax;
  int32_t window;
  int32_t n_replay;     /* > 0: replay these segments instead of adapting    */
  const double* replay; /* host, n_replay x (t_start, h, n_steps)             */
  double* record;       /* host, record_cap x (t_start, h, n_steps), or NULL  */
  int32_t record_cap;
  int32_t compensated;  /* AQC_C64: 1 (recommended) keeps the state as a
                           pair hi + lo updated by exact two-sums, hi in the
                           caller's complex64 psi and lo (the rounding
                           residual) as a bfloat16 pair in the workspace, so
                           rounding of the stored state does not accumulate
                           (half a state vector of workspace and of traffic
                           read and written per step); 0 stores y in
                           complex64 only.  Ignored for AQC_C128.             */
  aqc_pc4_carry* carry; /* fixed-step pc4 only: continue / start a chain, or
                           NULL for a self-contained call                     */
} aqc_evolve_opts;

typedef struct {
  int64_t steps;        /* accepted steps                                     */
  int64_t rejected;     /* steps undone by the adaptive controller            */
  int64_t matvecs;      /* evaluations of H|psi>                              */
  int32_t n_segments;   /* segments written to opts.record (or needed)        */
  int32_t status_step;  /* step at which the guard tripped (-1 if none)       */
  double t_reached;
  double h_last;
  double shift_used;
  double rho;           /* half-width of the enclosure after the shift       */
  double norm2_initial;
  double norm2_final;
  double max_err;       /* largest Milne estimate of accepted pc4 steps      */
} aqc_evolve_stats;

/* Bytes of device workspace aqc_evolve needs for this Hamiltonian and dtype:
 * 5 state vectors for pc4, 2 for rk4, one more when H|psi> takes several
 * tile passes, one more when the last pass has stream groups (a second y^p),
 * half a vector for a compensated complex64 state, and for the adaptive
 * controller's checkpoint one vector (and half a vector when compensated).  */
size_t aqc_evolve_workspace_bytes(const aqc_ham* ham, int dtype, const aqc_evolve_opts* opts);

/* aqc_evolve: psi holds psi(t0) on entry and psi(t1) on return (in place).
 * Solves i d psi/dt = H(t) psi (eq. (schroedinger)) on the grid
 * t_k = t_start + k h of each segment.  pc4: three RK4 steps start every
 * segment, then one H|psi> per step.  A constant shift c is subtracted from H
 * and exp(-i c (t1 - t0)) is multiplied back in at the end.  Synchronous: the
 * statistics are final on return.  EUNSTABLE: the norm guard tripped or
 * h * rho > stab_limit; psi then holds the last state reached and
 * stats->t_reached says when.  ENOMEM: ws_bytes too small.                  */
aqc_status aqc_evolve(aqc_ctx* ctx, const aqc_ham* ham, void* psi, int dtype, double t0,
                      double t1, const aqc_evolve_opts* opts, void* workspace,
                      size_t ws_bytes, aqc_evolve_stats* stats);

/* ---- reductions (float64) ---------------------------------------------- */
/* sum_z |psi_z|^2 */
aqc_status aqc_norm2(aqc_ctx* ctx, const void* psi, int dtype, int n_qubits, double* out);
/* <phi|psi> = sum_z conj(phi_z) psi_z */
aqc_status aqc_overlap(aqc_ctx* ctx, const void* phi, const void* psi, int dtype,
                       int n_qubits, double* re, double* im);

#define AQC_TARGET_STATE      0  /* target: device state |phi>; |<phi|psi>|^2   */
#define AQC_TARGET_BASIS_LIST 1  /* target: host int64 list of basis states;
                                    sum of |psi_z|^2 over the distinct entries  */
/* Success probability P_1 (Sec. III.B). */
aqc_status aqc_fidelity(aqc_ctx* ctx, const void* psi, int dtype, int n_qubits,
                        int target_kind, const void* target, int64_t target_len,
                        double* out);
/* Mass of psi on the ground set of the diagonal part of H(t):
 * {z : E(z) <= E_min + rel_tol * max(1, |E_min|)}; also returns E_min.  For a
 * problem Hamiltonian with a unique solution this is P_1(T) (Sec. III.B).   */
aqc_status aqc_ground_mass(aqc_ctx* ctx, const aqc_ham* ham, double t, const void* psi,
                           int dtype, double rel_tol, double* mass, double* e_min);
/* <psi|H(t)|psi> (real), the energy E(T) of Sec. III.B.  Workspace as for
 * aqc_apply.                                                                */
aqc_status aqc_energy(aqc_ctx* ctx, const aqc_ham* ham, double t, const void* psi,
                      int dtype, void* workspace, size_t ws_bytes, double* out);
/* aqc_energy for callers that cannot allocate device memory (code that is
 * being captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc): the same value from the same kernels, but the partial product
 * of the high passes and the per-workgroup partial sums live in a fixed
 * device array of the library (32 MiB + 1 MiB, one copy per GPU, held until
 * the process ends) instead of a caller workspace and the context's
 * reduction buffer.  No workspace argument; no hipMalloc, hipFree or other
 * allocation.  Limits: the partial product fits states of up to 2^22
 * complex64 or 2^21 complex128 amplitudes (single-pass plans, n <= 13 or 12,
 * need none), and at most 43690 last-pass workgroups; larger problems return
 * AQC_ENOMEM with the sizes in the message.  The Hamiltonian's plan for this
 * dtype must exist: it is built with the Hamiltonian up to 26 qubits (and
 * rebuilt by aqc_ham_set_tiling), otherwise by a first aqc_apply or
 * aqc_energy call; AQC_EINVAL if not.  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one device (two host threads,
 * or two streams) race and give wrong results; the array keeps the last
 * call's contents, none of which a call reads before writing.  Synchronises
 * the context's stream.                                                     */
aqc_status aqc_energy_noalloc(aqc_ctx* ctx, const aqc_ham* ham, double t, const void* psi,
                              int dtype, double* out);
/* aqc_norm2 and aqc_overlap on states of `len` amplitudes (sector states).  */
aqc_status aqc_norm2_len(aqc_ctx* ctx, const void* psi, int dtype, int64_t len, double* out);
aqc_status aqc_overlap_len(aqc_ctx* ctx, const void* phi, const void* psi, int dtype,
                           int64_t len, double* re, double* im);

/* ---- Hamming-weight sectors (Sec. III.A.2-3, eq. (Sigmaz)) ---------------- */
/* H^xyz (eq. (Hixyz)), H^xy (eq. (Hixy)) and a diagonal H_f commute with
 * Sigma^z, so the number w of 1-bits of the basis states is conserved and a
 * solve started in the sector of weight w (e.g. from eq. (initstate)) never
 * leaves it.  aqc_sector_create restricts `ham` to that sector: a state of the
 * result holds the C(n, w) amplitudes of the weight-w basis states in
 * increasing order of z, i.e. amplitude r belongs to the z whose set bits
 * p_0 < p_1 < ... have sum_k C(p_k, k + 1) = r.  The result is an aqc_ham
 * accepted, on such states, by aqc_apply, aqc_apply_workspace_bytes,
 * aqc_evolve (every method and option, pc4 chains included),
 * aqc_evolve_workspace_bytes, aqc_energy, aqc_ground_mass (mass on the lowest
 * diagonal energies within the sector) and aqc_spectral_bounds (enclosure of
 * the sector's spectrum); not by aqc_batch_admit (AQC_ENOTSUP) or
 * aqc_ham_set_tiling (AQC_EINVAL); free it with aqc_ham_free.  It copies what
 * it needs: `ham` may be freed first.
 * Requirements, else AQC_EINVAL: 0 <= weight <= n; every off-diagonal term
 * flips exactly two bits, and for each such pair and schedule the summed
 * coefficient vanishes on the states whose two bits are equal (checked
 * exactly over the terms' Z bits, at most 16 besides the pair, else
 * AQC_ENOTSUP).  n <= 34, at most 600 flip pairs and 1024 pair terms
 * (AQC_ENOTSUP).
 * Device tables: a few tens of KB, allocated here.  When the diagonal terms
 * use at most two schedules and 8 C(n, w) bytes per schedule come to at most
 * 16 GiB, the diagonal is also kept per state, split by schedule (float64,
 * computed here on the context's stream, which is synchronised): products
 * then read it instead of summing the terms per state.                     */
aqc_status aqc_sector_create(aqc_ctx* ctx, const aqc_ham* ham, int weight, aqc_ham** out);
/* amplitudes of a state of `ham`: 2^n, or C(n, w) for a sector            */
int64_t aqc_ham_dim(const aqc_ham* ham);
/* the sector's weight, or -1 for a full-space Hamiltonian                  */
int aqc_ham_sector_weight(const aqc_ham* ham);
/* psi_full (2^n amplitudes, caller-owned device memory) = psi_s placed at
 * its basis states, zero elsewhere; the two must not overlap.              */
aqc_status aqc_sector_expand(aqc_ctx* ctx, const aqc_ham* sector, const void* psi_s,
                             void* psi_full, int dtype);
/* psi (C(n, w) amplitudes) = the balanced superposition of eq. (initstate),
 * every amplitude C(n, w)^{-1/2}.                                          */
aqc_status aqc_sector_dicke(aqc_ctx* ctx, const aqc_ham* sector, void* psi, int dtype);

/* ---- lowest eigenvalues (Sec. IV.B) ---------------------------------------- */
/* The n_eig (1..8) smallest eigenvalues of H(t) (a full-space Hamiltonian or
 * a sector), for the lower spectrum and the gap E_1 - E_0 along a path that
 * the paper computes with ARPACK.  Thick-restart Lanczos with full
 * reorthogonalisation (classical Gram-Schmidt twice) in a basis of
 * max_basis (n_eig + 2 .. 48, at most the dimension) vectors; each restart
 * keeps min(max_basis - 2, max(n_eig + 4, 2 n_eig)) Ritz vectors.  Products,
 * dot products and updates run on the device (float64 sums); the projected
 * matrix is diagonalised on the host.  Converged when every residual
 * ||H x_i - theta_i x_i|| <= tol * max(1, |theta_i|); complex64 bases reach
 * about 1e-6 relative, complex128 about 1e-13.  A level of multiplicity > 1
 * may be reported once: one Krylov sequence sees one vector of each
 * eigenspace (exactly so for a diagonal H).
 * start: a device state (copied, normalised) or NULL for a fixed
 * pseudo-random start.  workspace: aqc_lowest_eigs_workspace_bytes; the
 * caller owns it.  Outputs: evals[n_eig] ascending, resid[n_eig], *matvecs,
 * and, when ground_out is not NULL, the normalised Ritz vector of evals[0]
 * (a device state of the Hamiltonian's dimension, e.g. the ground state of
 * H^xy in a sector that starts the XY algorithm, Sec. III.A.3).
 * AQC_EUNSTABLE when max_matvecs products did not converge (the outputs then
 * hold the last Ritz values); AQC_EINVAL on bad sizes or a zero start.      */
aqc_status aqc_lowest_eigs(aqc_ctx* ctx, const aqc_ham* ham, double t, int dtype, int n_eig,
                           int max_basis, int max_matvecs, double tol, const void* start,
                           void* workspace, size_t ws_bytes, double* evals, double* resid,
                           int* matvecs, void* ground_out);
size_t aqc_lowest_eigs_workspace_bytes(const aqc_ham* ham, int dtype, int max_basis);
/* Host-only: eigenvalues (ascending, w[n]) and optionally eigenvectors
 * (columns of z, interleaved re/im, row-major n x n) of a Hermitian matrix a
 * (interleaved re/im, row-major n x n, n <= 512) by cyclic Jacobi rotations;
 * the solver of the projected Lanczos problem.  Needs no device.            */
aqc_status aqc_hermitian_eigh(int n, const double* a, double* w, double* z);

/* ---- batches of solves ------------------------------------------------------ */
/* A batch advances many independent fixed-step predictor-corrector solves
 * (each its own Hamiltonian, n, interval, step and shift) together: every
 * "tick" performs one H|psi> per active solve, with one launch per tile-pass
 * level for all solves (the workgroups of a launch are mapped to (solve, tile)
 * pairs).  Each solve runs exactly the launch sequence aqc_evolve uses for
 * {AQC_METHOD_PC4, n_steps, AQC_SHIFT_VALUE shift, compensated}, so its result
 * does not depend on what else is in the batch.  The batch works on its own
 * stream, ordered after and before the context's stream by events; with
 * graphs on, each tick is replayed as a captured hipGraph (re-captured when
 * the set of active solves changes).  States and workspaces stay owned by the
 * caller and must stay allocated until the solve is retired.               */
typedef struct aqc_batch aqc_batch;
aqc_status aqc_batch_create(aqc_ctx* ctx, int dtype, int capacity, aqc_batch** out);
/* aqc_batch_destroy: waits for the batch's streams (and for the context's
 * stream while the context lives), frees the batch and drops its hold on the
 * context.                                                                  */
aqc_status aqc_batch_destroy(aqc_batch* batch);
aqc_status aqc_batch_set_graph(aqc_batch* batch, int on);
/* Resident solves.  With max_n > 0 (at most 20), a solve admitted later with
 * n <= max_n is not stepped by the ticks: the next aqc_batch_step launches
 * all such solves admitted since the previous step in one persistent launch,
 * one workgroup per solve, which runs each solve's whole fixed-step pc4
 * segment (RK4 bootstrap, predictor-corrector steps, the shift's phase) with
 * workgroup barriers only, on a stream of the batch, ordered after the
 * context stream's earlier work.  It uses the Hamiltonian's plan of tile
 * passes only (built on first use), so its results equal aqc_evolve's to
 * rounding, not bit for bit.  Such a solve counts as running until its launch
 * has finished; aqc_batch_poll reports it then, and aqc_batch_step, when it
 * has no ticks to run, waits for the oldest resident launch instead of
 * returning at once.  Plans that do not fit (more than four passes, a tile
 * larger than the LDS) fall back to the ticks.  0 (the default) turns it off.
 * EINVAL for max_n outside 0..20.                                           */
aqc_status aqc_batch_set_resident(aqc_batch* batch, int max_n);
/* workspace one solve needs (pc4, compensated for AQC_C64)                   */
size_t aqc_batch_workspace_bytes(const aqc_ham* ham, int dtype);
/* Admit the solve psi(t0) -> psi(t1) in n_steps equal steps with the constant
 * shift; psi is evolved in place.  EBUSY when every slot is taken.           */
aqc_status aqc_batch_admit(aqc_batch* batch, const aqc_ham* ham, void* psi, void* workspace,
                           size_t ws_bytes, double t0, double t1, int64_t n_steps, double shift,
                           int* slot);
/* Run up to `ticks` ticks (fewer when every solve has finished); returns the
 * number of solves still running.                                           */
aqc_status aqc_batch_step(aqc_batch* batch, int ticks, int* n_active);
/* Finished solves not reported before (their psi holds psi(t1) once this
 * returns: it synchronises the batch stream).                               */
aqc_status aqc_batch_poll(aqc_batch* batch, int* slots, int cap, int* n_done);
/* Release a finished slot; fills steps, matvecs, t_reached, h_last, shift.   */
aqc_status aqc_batch_retire(aqc_batch* batch, int slot, aqc_evolve_stats* stats);
aqc_status aqc_batch_info(const aqc_batch* batch, int* active, int* finished, int64_t* ticks);

/* ---- instrumentation ----------------------------------------------------- */
/* Kernel timing with HIP events recorded on the context's stream around every
 * tile-pass launch (the events add no synchronisation).  Classes:
 *   AQC_PROF_HIGH_PASS  passes that apply high-qubit flips and write the partial
 *                       product;
 *   AQC_PROF_LAST_PASS  the last pass: diagonal, low flips and the fused stage
 *                       update.
 * aqc_profile_read synchronises the stream and returns the summed kernel time
 * (ms), the number of launches and their algorithmic bytes (each vector a
 * launch must read or write, counted once: the tile source, the partial
 * product in and out, and the stage update's streamed inputs and outputs)
 * since the last reset.                                                     */
#define AQC_PROF_HIGH_PASS 0
#define AQC_PROF_LAST_PASS 1
aqc_status aqc_profile_enable(aqc_ctx* ctx, int on);
aqc_status aqc_profile_reset(aqc_ctx* ctx);
aqc_status aqc_profile_read(aqc_ctx* ctx, int kind, double* total_ms, int64_t* launches,
                            double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* AQC_H */
