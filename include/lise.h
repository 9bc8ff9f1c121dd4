/*
 * lise.h - C-ABI of the MI355X (gfx950) TDSLDA time-step library.
 *
 * The library evolves a set of quasiparticle wavefunctions (qpwfs) on a
 * periodic 3D lattice under the time-dependent superfluid local density
 * approximation of arXiv:2009.00745 (Sec. "Time-dependent superfluid local
 * density approximation", Eq. tdslda), with the kinetic operator taken by FFT
 * (Sec. "Discretization"), the local mean field U and pairing field Delta
 * rebuilt from the densities of Eq. (rho_t, nu_t) and Eq. (pairingfield), and
 * the Adams-Bashforth-Milne predictor-modifier-corrector of Sec. "Time
 * evolution", Eq. (p), (m), (c), (y), started by the series-expansion
 * predictor-corrector of the same section.
 *
 * Conventions
 *   - hbar = m = 1.  Lattice spacing a on all three axes; x is the fastest
 *     index.  Lattice points N = nx*ny*nz.  Qpwf j, component c, point
 *     (z, y, x) lives at element ((j*C + c)*nz + z)*ny*nx + y*nx + x.
 *   - C = 2 components are (u, v) = the (u_up, v_dn) block of Eq. tdslda;
 *     C = 4 components are (u_up, u_dn, v_up, v_dn).
 *   - Host-side qpwf and field data are complex128 (interleaved re, im) or
 *     float64, whatever the internal precision; the library converts.
 *   - Every call enqueues its work on the context's HIP stream (the stream
 *     given to lise_init / lise_set_stream, e.g. PyTorch's current stream).
 *     Calls that return host data synchronise that stream before returning.
 *   - The context owns every device buffer it allocates; pointers passed by
 *     the caller are borrowed for the duration of the call only.
 *   - A context is not thread-safe; use one context per host thread.
 *   - Return value: LISE_OK (0) or a negative LISE_E_* code.  The message of
 *     the last error is available from lise_last_error(ctx).  No exception
 *     crosses the ABI.
 */
#ifndef LISE_H
#define LISE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LISE_OK 0
#define LISE_E_ARG (-1)          /* invalid argument (null pointer, range, size) */
#define LISE_E_NOMEM (-2)        /* device or host allocation failed */
#define LISE_E_UNSUPPORTED (-3)  /* lattice/precision not supported (e.g. a prime factor > 5) */
#define LISE_E_HIP (-4)          /* a HIP runtime call or kernel launch failed */
#define LISE_E_STATE (-5)        /* call out of order (e.g. stepping before qpwfs are set) */
#define LISE_E_NAN (-6)          /* non-finite value detected in the densities */

typedef struct lise_ctx lise_ctx;

/* Periodic lattice of nx*ny*nz points with spacing a (Sec. Discretization:
 * x_n = n a, n = 0..N-1; momenta k_n = 2 pi n / L for n < N/2 and
 * 2 pi (n - N) / L otherwise, L = N a).  Each of nx, ny, nz must factor into
 * 2, 3 and 5 only and lie in [1, 128].  In addition one xy-plane of both
 * components of a pair must fit the plane kernel: square planes of side 8,
 * 16, 20, 24, 32, 48 or 64 always do; other planes need nx*ny <= 2560 points
 * (LISE_FP64) or <= 4096 (LISE_FP32), and an nz x nx tile must fit the
 * z-axis kernel (nz*nx <= 5120 for LISE_FP64, 10240 for LISE_FP32, unless nz
 * is one of the sides above).  lise_init returns LISE_E_UNSUPPORTED
 * otherwise.  (LISE_FP64 planes of side 64 run with register spills: a
 * 64-point line over 16 lanes leaves 128 registers per thread.) */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;
    double a;
} lise_lattice;

/* Arithmetic of the state, FFTs and integrator.  Densities, potentials,
 * norms and energies are always accumulated in float64. */
typedef enum {
    LISE_FP64 = 0,       /* complex128 state */
    LISE_FP32 = 1,       /* complex64 state, float64 sums */
    LISE_FP32_MFMA = 2,  /* as LISE_FP32, with the xy-plane kinetic term as two
                            dense products with the DVR kinetic matrix on the
                            matrix cores, operands split into bf16 hi + lo
                            (three products, float32 accumulation); square
                            xy-planes of side 16, 32, 48 or 64 only */
} lise_precision;

/* Functional and Hamiltonian parameters.
 *   U(r)     = beta * n(r)^(2/3)   (self-consistent mean field)
 *   Delta(r) = -g * kappa(r)       (Eq. pairingfield)
 *   V(r, t)  = U(r) + U_ext(r, t), h = T + V (T = -Laplacian/2 by FFT)
 *   U_ext    = ext_A * ramp(t) * exp(-d^2 / (2 ext_w^2)), d = minimum-image
 *              distance to ext_r0 (Sec. "External boosts and external
 *              potentials"); ramp = sin^2(pi t / (2 ext_t_on)) for
 *              0 <= t < ext_t_on, else 1.
 * C = 2 densities: n = w sum_j |v_j|^2, kappa = (w/2) sum_j v_j^* u_j.
 * C = 4 densities (Eq. rho_t, nu_t, singlet average):
 *   n = sum_j (|v_up|^2 + |v_dn|^2), kappa = 1/2 sum_j (v_dn^* u_up - v_up^* u_dn).
 * frozen = 1 replaces U and Delta by the constants U0 and Delta0 (test mode).
 * regularize = 1 replaces g by the lattice-renormalised coupling of
 * Eq. (geff_3D) for a cubic lattice with its natural cutoff (m* = m = 1):
 *   1/g_eff = 1/g - K / (4 pi a),
 *   K = (12/pi) int_0^{pi/4} ln(1 + 1/cos^2 t) dt = 2.44274960780633...
 * in Delta and in E_pair; regularize = 0 keeps the bare g.
 * remove_phase = 1 evolves every qpwf with H - eta_j instead of H
 * (Eq. sp_en), eta_j = <psi_j|H|psi_j> = a^3 sum_r sum_c psi_c^* (H psi)_c
 * of the vector H acts on, taken in every right-hand side: y'_n and m' of
 * the ABM step, and in each series-expansion start-up step
 * exp(-i dt (H_s - eta)) with eta from psi_s and the H of that
 * propagation.  It removes the trivial phase of Eq. (phase) and leaves the
 * densities unchanged up to the integration error.  Costs one more plane
 * pass per H application (measured 1.08x the step at 32^3 FP64). 
 * C = 2 uses mu_up as its single chemical potential. */
typedef struct {
    int32_t ncomp;          /* 2 or 4 */
    int32_t precision;      /* lise_precision */
    double mu_up, mu_dn;
    double beta, g, w;
    int32_t frozen;
    int32_t regularize;     /* 0 or 1, see above */
    double U0, Delta0_re, Delta0_im;
    double ext_A, ext_w;
    double ext_r0[3];
    double ext_t_on;
    int32_t remove_phase;   /* 0 or 1, see above */
    int32_t reserved;       /* must be 0 */
} lise_functional;

/* Observables of the current state (Sec. "Miscellaneous quantities" and the
 * cold-atom energy):
 *   N = a^3 sum_r n;  E = E_kin + E_int + E_pair + E_ext with
 *   E_kin  = a^3 sum_r weight * sum_j Re(v_j^* T v_j)  (same T as the step),
 *   E_int  = a^3 sum_r (3/5) beta n^(5/3),  E_pair = a^3 sum_r g |kappa|^2,
 *   E_ext  = a^3 sum_r U_ext n;
 *   mean_abs_delta = sum |Delta| n / sum n;  r_cm = sum r n / sum n;
 *   norm_drift_* = max / mean over j of |<psi_j|psi_j> - <psi_j|psi_j>_0|,
 *   relative to the norms when the qpwfs were last set;
 *   P = a^3 sum_r j(r) with j of lise_current, v_cm = P / N.  With the
 *   register-FFT kernels on all axes (square planes and sides of 8, 16, 20,
 *   24, 32, 48 or 64) P is formed from Parseval sums of the same spectral
 *   derivatives instead of the field (equal to rounding).
 *   N_up, N_dn: the spin-resolved terms of Eq. (rho_t), N_sigma = a^3 sum_r
 *   sum_j |v_{j,sigma}|^2 (C = 4: components v_up, v_dn); the C = 2 reduction
 *   is spin-symmetric by construction (each state of the (u_up, v_dn) block
 *   stands for itself and its time-reversed partner), N_up = N_dn = N / 2. */
typedef struct {
    double t;
    int64_t step;
    double N, E, E_kin, E_int, E_pair, E_ext;
    double mean_abs_delta;
    double r_cm[3];
    double norm_drift_max, norm_drift_mean;
    double P[3];      /* a^3 sum_r j (total current of Eq. j) */
    double v_cm[3];   /* P / N (Eq. vel, m = hbar = 1) */
    double N_up, N_dn;
} lise_obs;

/* Launch tuning (0 = library default).
 *   chunk_qpwf : qpwfs per launch of the two apply-H kernels; sizes the
 *                z-term scratch (chunk x C x N elements, a second one when
 *                the z kernel overlaps; default: about 4 GiB of qpwfs)
 *   jgroup     : qpwfs that one workgroup of the plane kernel walks through
 *                (sets the number of density partial sums; 0 = default:
 *                32, 16 on the single-pass path and 128 on the z_dense path
 *                below)
 *   fused      : whole-cube kernel (one pass, the cube in LDS): 1 = whenever
 *                the cube fits in LDS; 0 = only where the register-FFT
 *                kernels below do not cover the lattice; -1 = never (always
 *                the z-axis kernel plus the plane kernel)
 *   generic    : 1 = use the runtime-sized LDS FFT kernels even where a
 *                size-specialised register-FFT kernel exists (sides 8, 16,
 *                20, 24, 32, 48, 64; square xy-planes for the plane kernel)
 *   no_overlap : 1 = run the z-axis kernel on the context stream; 0 = run it
 *                one chunk ahead on an internal stream of default priority
 *                (two z-scratch buffers, ordered by events)
 *   graph      : 1 = lise_step captures four ABM steps (one period of the
 *                buffer ring) in a HIP graph and replays it; results are
 *                bit-identical to eager stepping
 *   single_pass: the ABM phases of cubic lattices of side 8 or 16 (and 20 in
 *                LISE_FP32) without phase removal run one kernel per phase
 *                that holds the whole component pair of a qpwf in LDS and
 *                applies the kinetic term as a 3D transform, instead of the
 *                z-axis kernel plus the plane kernel (no z-term scratch: 14
 *                state arrays per step instead of 20; at side 20 and in
 *                float64 at side 16 the densities take a pass of their
 *                own, 16 arrays).  1 = wherever available, 0 = default
 *                (side 8, and 16 and 20 in LISE_FP32: measured faster there
 *                than the two kernels; float64 at 16 slower), -1 = never;
 *                start-up, lise_apply_h and the observables keep the two
 *                kernels.  jgroup's default is 16 qpwfs per workgroup on
 *                this path (32 on the others).  lise_autotune times both
 *                paths.
 *   z_lanes    : lanes that share one z-column in the register-FFT z-axis
 *                kernel: 1 (the column in one thread's registers), 2 or 4
 *                (each lane nz/L points, exchanges across lanes); 0 =
 *                default (1); a value that does not divide nz into >= 2
 *                points per lane falls back to 1.  Errors: ARG for other
 *                values.
 *   z_dense    : the ABM phases compute the z-term inside the plane kernel,
 *                as the dense real symmetric nz x nz matrix T_z applied to
 *                the z-columns of the input, instead of running the z-axis
 *                kernel and reading its scratch back (no z-term scratch: 14
 *                state arrays per step from HBM when the columns of a qpwf
 *                stay in L2 while its planes are processed; one workgroup
 *                takes 4 planes, the workgroups of one qpwf group are
 *                launched onto one XCD, and one launch covers all qpwfs).
 *                Available on cubic lattices of side 32 (float64 and
 *                float32) and 16 (float64) on the register-FFT kernels, off
 *                the single-pass path, without phase removal.  1 = on where
 *                available, 0 = default (on for float64 side 32, where it
 *                measured faster than the two kernels; float32 measured
 *                slower), -1 = off.  jgroup's default is 128 on this path.
 *                Results agree with the two-kernel path to rounding (dense
 *                sums instead of transforms).  lise_autotune times both.
 *                Errors: ARG for other values.  A context on this path is
 *                stepped alone by lise_batch_step. */
typedef struct {
    int32_t chunk_qpwf;
    int32_t jgroup;
    int32_t fused;
    int32_t generic;
    int32_t no_overlap;
    int32_t graph;
    int32_t single_pass;
    int32_t z_lanes;
    int32_t z_dense;
} lise_tuning;

/* Create a context for n_qpwf qpwfs on `lat` with functional `fn`, on the
 * HIP stream `hip_stream` (hipStream_t; NULL = the null stream).  Allocates
 * the seven state copies of the ABM history (y_n, y_{n-1}, four derivative
 * levels, p - c) plus scratch.  The qpwfs are undefined until lise_set_qpwf
 * has covered all of them.  Errors: ARG, UNSUPPORTED, NOMEM, HIP. */
int lise_init(lise_ctx **out, const lise_lattice *lat, int64_t n_qpwf,
              const lise_functional *fn, void *hip_stream);

/* Copy qpwfs [first, first+count) from `src` (complex128, count*C*N
 * elements, layout above) into the state; `src_is_device` = 1 when src is a
 * device pointer.  Keeps the time (see lise_set_time), discards the ABM
 * history, and marks densities stale.  The context records which qpwfs have
 * been written: every call that needs the whole state (lise_step,
 * lise_startup, lise_apply_h, lise_densities, lise_observables, lise_save,
 * lise_kick, lise_current, lise_autotune, lise_batch_step) returns
 * LISE_E_STATE until each of the M qpwfs has been covered by some call since
 * the last reset.  Resets: context creation, a failed lise_load, and the
 * first lise_set_qpwf after the state was evolved (the evolved qpwfs no
 * longer sit where a partial update would leave them).
 * Errors: ARG, STATE, HIP. */
int lise_set_qpwf(lise_ctx *c, int64_t first, int64_t count, const void *src, int32_t src_is_device);

/* Copy qpwfs [first, first+count) of the current state y_n to `dst`
 * (complex128).  Errors: ARG, HIP. */
int lise_get_qpwf(lise_ctx *c, int64_t first, int64_t count, void *dst, int32_t dst_is_device);

/* H psi (Eq. tdslda, with h = T + V, h_updn = 0) for qpwfs [first,
 * first+count) of the current state, with U and Delta built from the
 * densities of the whole current state at the current time.  `out` receives
 * count*C*N complex128 values (device pointer if out_is_device = 1, else
 * host).  Errors: ARG, STATE, HIP. */
int lise_apply_h(lise_ctx *c, int64_t first, int64_t count, void *out, int32_t out_is_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): lise_apply_h with
 * a device output that calls no hipMalloc, hipFree or allocating routine.
 * `out_device` receives count*C*N complex128 values (caller-owned device
 * memory).  H psi is staged, in pieces, through one fixed device array of
 * LISE_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the
 * process ends (lise_apply_h instead allocates a staging buffer of its own at
 * its first call); results equal lise_apply_h bit for bit.  The array is
 * shared by every context and call on that GPU and keeps the last call's
 * contents: calls that overlap on one GPU (different streams or host
 * threads) race.  The context, its fields and z-term scratch are allocated
 * by lise_init, before.  Errors: ARG, STATE, UNSUPPORTED (one qpwf, C*N
 * elements of the state's precision, larger than the array), HIP. */
#define LISE_NOALLOC_SCRATCH_BYTES (64 << 20)
int lise_apply_h_noalloc(lise_ctx *c, int64_t first, int64_t count, void *out_device);

/* Series-expansion start-up (Sec. "Time evolution"): three predictor-
 * corrector steps of order 4 with corrector densities (n_pre + n)/2 taken at
 * t + dt/2; stores y'_0, y'_1, y'_2 = -i H y_s, y_2, y_3 and p_3 - c_3 = 0.
 * Advances t by 3 dt.  Errors: STATE, HIP, NAN. */
int lise_startup(lise_ctx *c, double dt);

/* Advance `nsteps` ABM steps (Eq. p, m, c, y; predictor coefficient of
 * y'_n = 119).  Runs lise_startup first when there is no history or when dt
 * differs from the history's step.  Per step: apply H to y_n, form p and m,
 * rebuild n, kappa, U, Delta from m at t + dt, apply H to m, form c and
 * y_{n+1}, rebuild the fields from y_{n+1}.  Errors: STATE, HIP, NAN. */
int lise_step(lise_ctx *c, double dt, int64_t nsteps);

/* Densities of the current state: n (N float64) and kappa (N complex128,
 * interleaved).  Either pointer may be NULL.  Errors: ARG, STATE, HIP. */
int lise_densities(lise_ctx *c, double *n_out, double *kappa_out, int32_t out_is_device);

/* Observables of the current state (see lise_obs).  Errors: ARG, STATE, HIP. */
int lise_observables(lise_ctx *c, lise_obs *out);

/* Current time and number of steps taken (start-up steps count). */
int lise_get_time(const lise_ctx *c, double *t, int64_t *step);

/* Set the time of the current state (before stepping). Errors: ARG. */
int lise_set_time(lise_ctx *c, double t);

/* Replace the stream all later work is enqueued on. */
int lise_set_stream(lise_ctx *c, void *hip_stream);

/* Override launch tuning (see lise_tuning).  Reallocates scratch as needed.
 * Errors: ARG, NOMEM. */
int lise_set_tuning(lise_ctx *c, const lise_tuning *t);

/* Per-kernel timing with HIP events on the context's stream.
 * lise_profile(c, 1) starts recording an event pair around every launch of
 * the library's kernels; lise_profile(c, 0) stops.  lise_profile_read
 * synchronises, then returns for kernel class `which` (0 = plane kernel of
 * ABM phase 1, 1 = z-axis kernel, 2 = density reduction + potentials,
 * 3 = plane kernel outside the ABM phases: start-up, apply-H, energy,
 * 4 = plane kernel of ABM phase 2) the
 * number of launches and their summed duration in milliseconds, and clears
 * that class's counters.  Returns LISE_E_STATE if more than 8192 launches
 * were recorded since the previous read (the event pool is fixed). */
int lise_profile(lise_ctx *c, int32_t enable);
int lise_profile_read(lise_ctx *c, int32_t which, int64_t *launches, double *total_ms);

/* Timed search over launch tuning for this system: chunk size (1/4, 1, 2 and
 * 4 GiB of qpwfs), qpwfs per plane workgroup 8/16/32/64 and z-kernel overlap
 * on the two-kernel path, 2/4/8/16 qpwfs per workgroup on the single-pass
 * path and 32/64/128/256 on the in-kernel z-term path where those apply (not
 * where the tuning turned them off); each candidate runs one untimed and
 * `trial_steps` timed ABM
 * steps with step size dt on the live state (the state advances; results
 * change only in rounding).  The three fastest run again over
 * 2 * trial_steps, each two-kernel one also with 2 and 4 lanes per z-column,
 * and the fastest of that round is kept and written to *chosen (may be
 * NULL).  Runs the start-up first if needed.  Errors: ARG, STATE, HIP, NAN. */
int lise_autotune(lise_ctx *c, double dt, int32_t trial_steps, lise_tuning *chosen);

/* Checkpoint and restart (Sec. "Checkpoint and restart").
 * lise_save writes the current state to the file `path` (created or
 * truncated).  with_history = 0 saves the latest qpwfs only, as the paper
 * does: a context that loads such a file restarts with the series-expansion
 * start-up at its next lise_step.  with_history = 1 (allowed once the ABM
 * history exists, i.e. after lise_startup or lise_step) also saves y_{n-1},
 * y'_{n-1}, y'_{n-2}, y'_{n-3}, p_n - c_n and the densities of y_n, so that
 * load + lise_step continues bit for bit as if never interrupted.
 * File layout, little-endian: a 112-byte header
 *   char magic[8] = "LISECKP1"; int32 version = 1, ncomp, precision, nx, ny,
 *   nz, history, elem_bytes (16 = complex128, 8 = complex64); float64 a;
 *   int64 M; float64 t; int64 step; float64 dt (0 without history);
 *   int64 reserved[4]
 * then arrays of M*C*N complex numbers of elem_bytes each, in the element
 * order of lise_set_qpwf: y_n; with history y_{n-1}, y'_{n-1}, y'_{n-2},
 * y'_{n-3}, p_n - c_n and 3N float64 (n, Re kappa, Im kappa of y_n); last M
 * float64 reference norms (the norms when the qpwfs were set).
 * lise_load reads such a file into a context created with the same lattice,
 * C, M and precision (else ARG) and restores t and the step count.  Both
 * calls synchronise the context stream and stage through pinned host memory.
 * Errors: ARG (path, file content, I/O), STATE (save before the qpwfs are
 * set, or history requested without one), HIP, NOMEM.  A failed load leaves
 * the context requiring lise_set_qpwf. */
int lise_save(lise_ctx *c, const char *path, int32_t with_history);
int lise_load(lise_ctx *c, const char *path);

/* Boost of Eq. (kick): u -> exp(i chi) u and v -> exp(-i chi) v for every
 * qpwf (C = 2: u = component 0, v = 1; C = 4: u_up, u_dn = 0, 1 and
 * v_up, v_dn = 2, 3).  chi holds N float64 in the lattice order (x fastest),
 * a host or device pointer (chi_is_device).  chi = p.r with p on the
 * momentum grid gives the system the velocity p.  The ABM history is
 * dropped: the next lise_step runs the start-up.
 * Errors: ARG, STATE (qpwfs not set), HIP. */
int lise_kick(lise_ctx *c, const double *chi, int32_t chi_is_device);

/* Current density of Eq. (j) of the current state,
 *   j(r) = -weight * sum_j Im(v_j^* grad v_j)
 * over the v components (C = 2: v with the weight w; C = 4: v_up, v_dn with
 * weight 1), with spectral first derivatives F^{-1}[i k F v] whose N/2 mode
 * (even axes) is zeroed, as the paper does for odd derivatives.  j_out: 3N
 * float64 (j_x, then j_y, then j_z, each in lattice order), host or device.
 * Errors: ARG, STATE, UNSUPPORTED (xy-plane above 4096 points or an xz-tile
 * that does not fit in LDS), HIP. */
int lise_current(lise_ctx *c, double *j_out, int32_t out_is_device);

/* The coupling g that Delta = -g kappa uses for this lattice and functional
 * (g itself, or g_eff when fn->regularize = 1), written to *g_out.  Host-only
 * arithmetic: needs no device and no context.
 * Errors: ARG (null pointer, regularize not 0/1, g = 0 or divergent g_eff). */
int lise_coupling(const lise_lattice *lat, const lise_functional *fn, double *g_out);

/* Batch of independent systems (for example different lattices and qpwf
 * counts) advanced together by the ABM step of Eq. (p), (m), (c), (y), each
 * under its own Eq. (tdslda) and densities (Sec. "Time evolution"; the batched
 * transforms of Sec. "FFT in batch").  lise_batch_create takes nsys distinct
 * contexts on the current device and moves all of them onto `hip_stream`;
 * the contexts stay owned by the caller and usable (densities, observables)
 * but must not be freed before the batch, nor stepped on their own while the
 * batch is in use (lise_batch_step notices and rebuilds its tables).
 *
 * lise_batch_step advances every system by nsteps ABM steps (start-up first
 * where a system has no history for dt).  Systems whose lattice the
 * register-FFT kernels cover (square xy-planes and z of side 8, 16, 20, 24,
 * 32, 48 or 64; LISE_FP64 or LISE_FP32; no phase removal; default kernels)
 * form groups of equal precision, xy side and z side.  Per ABM phase each
 * group runs one z-axis launch and one plane-kernel launch over all qpwfs of
 * all its systems (a device table holds one descriptor per system: buffers,
 * fields, functional, qpwf count and jgroup), then one launch rebuilds the
 * densities and fields of every grouped system and one more advances their
 * times.  With graphs on (the default) four steps, one period of the buffer
 * ring, are captured once on an internal stream as one graph of kernel
 * nodes and replayed on `hip_stream`; steps that do not fill a period run
 * eagerly.  The group's z-term scratch (sum over its systems of M*C*N
 * elements) is allocated by the first step.  Other systems are stepped one
 * after another on the same stream.  Results equal lise_step on each system
 * alone bit for bit when that system's chunk_qpwf covers all its qpwfs (the
 * default for up to about 1 GiB of qpwfs), since the density sums then run
 * in the same order.  Returns after all systems finished.
 * Errors: ARG, STATE, UNSUPPORTED (a group with more plane-kernel workgroup
 * rows than the device's grid allows), NOMEM, HIP, NAN (text from
 * lise_batch_last_error).
 *
 * lise_batch_set_graph: 1 (default) = replay captured periods, 0 = eager.
 * lise_batch_info: number of groups and of systems stepped one by one, as
 * of the last lise_batch_step (0, 0 before the first).
 * lise_batch_profile / lise_batch_profile_read: HIP-event timing of the
 * batch's launches, as lise_profile, for kernel class `which` (0 = plane
 * kernel of ABM phase 1, 1 = z-axis kernel, 2 = densities + fields, 3 =
 * plane kernel of ABM phase 2); steps run eagerly while profiling is on. */
typedef struct lise_batch lise_batch;
int lise_batch_create(lise_batch **out, int32_t nsys, lise_ctx *const *ctxs, void *hip_stream);
int lise_batch_step(lise_batch *b, double dt, int64_t nsteps);
int lise_batch_set_graph(lise_batch *b, int32_t enable);
int lise_batch_info(const lise_batch *b, int32_t *ngroups, int32_t *nsolo);
int lise_batch_profile(lise_batch *b, int32_t enable);
int lise_batch_profile_read(lise_batch *b, int32_t which, int64_t *launches, double *total_ms);
const char *lise_batch_last_error(const lise_batch *b);
void lise_batch_free(lise_batch *b);

/* Bytes of device memory the context holds. */
int lise_memory(const lise_ctx *c, int64_t *bytes);

/* Text of the last error on this context (never NULL). */
const char *lise_last_error(const lise_ctx *c);

/* Library version string. */
const char *lise_version(void);

/* Release every device buffer and the context.  NULL is a no-op. */
void lise_free(lise_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* LISE_H */
