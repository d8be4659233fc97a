/*
 * prs.h -- C ABI of the MI355X (gfx950) Press-Ryden-Spergel domain-wall
 * evolution library (libprs.so).
 *
 * The method is that of Correia & Martins, "General purpose graphics-
 * processing-unit implementation of cosmological domain wall network
 * evolution" (arXiv:1710.10420), Sec. II:
 *
 *   Eq. (1)  V(phi) = V0 (phi^2/phi0^2 - 1)^2
 *   Eq. (2)  phi'' + alpha (d ln a/d ln eta) phi'/eta - Lap phi = -a^beta dV/dphi,
 *            with the PRS choice beta = 0, alpha = 3 (the exact equations
 *            have alpha = beta = 2); a(eta) = (eta/eta0)^m
 *   Eq. (3)  Lap phi_i = sum_d (phi_{i+e_d} + phi_{i-e_d}) - 2 D phi_i   (/dx^2)
 *   Eq. (4)  phi_dot^{n+1/2} = [(1-delta) phi_dot^{n-1/2}
 *                               + deta (Lap phi^n - a_n^beta V'(phi^n))] / (1+delta)
 *   Eq. (5)  phi^{n+1} = phi^n + deta phi_dot^{n+1/2}
 *   Eq. (6)  delta = (1/2) alpha (deta/eta) (d ln a/d ln eta)
 *   Eq. (7)  rho = A/V: sum over sign-changing links of
 *            |grad phi| / (|phi_,x| + |phi_,y| + |phi_,z|), times dx^(D-1)/V
 *   Eq. (8)  (gamma v)^2 = (1/N) sum over wall sites of (1/2) phi_dot^2 / V(phi)
 *            (with beta != 0 the wall's potential energy a_n^beta V(phi))
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All functions are extern "C", never throw and return a prs_status.  On
 *   failure prs_last_error() holds a message (thread local).
 * - Fields are device arrays (HBM) of n[0]*n[1]*n[2] sites (n[2] = 1 in 2D),
 *   x fastest: site (x,y,z) is element x + nx*(y + ny*z), of float32 values
 *   (precision PRS_F32, the default) or float64 values (PRS_F64: the paper
 *   runs both precisions, Sec. III).  Boundaries are periodic.  Field
 *   pointers must be 16-byte aligned.  The caller owns every device buffer it
 *   passes; the library never frees them.
 * - All device work is enqueued on the caller's HIP stream (a hipStream_t
 *   passed as void*; NULL is the default stream).  Calls that return host
 *   results synchronise that stream before returning.
 * - The state after n steps is (phi^n, phi_dot^{n-1/2}); eta_n = eta0 + n*deta.
 * - Arguments are validated before any launch; invalid ones give PRS_EINVAL
 *   and leave every buffer untouched.  A failed HIP call gives PRS_EDEVICE.
 */
#ifndef PRS_H
#define PRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t prs_status;
#define PRS_OK 0
#define PRS_EINVAL (-1)        /* invalid argument (checked before any launch) */
#define PRS_ENOMEM (-2)        /* workspace too small or host allocation failed */
#define PRS_EDEVICE (-3)       /* a HIP runtime call failed */
#define PRS_ESTATE (-4)        /* call not valid in the object's current state */
#define PRS_EUNSUPPORTED (-5)  /* valid physics this library does not implement */

/* Run parameters (Sec. II).  V0 is derived as pi^2 / (2 W0^2), the height for
 * which the continuum kink tanh(pi x / W0) solves the static equation;
 * W0 = +inf gives V0 = 0 (free field). */
typedef struct prs_params {
    int32_t ndim;        /* 2 or 3 */
    int32_t diag_every;  /* K > 0: record diagnostics of every state n with
                            n % K == 0 (fused into step n); 0: none */
    int64_t n[3];        /* lattice sides nx, ny, nz (nz ignored in 2D), >= 1 */
    double dx;           /* lattice spacing, > 0 */
    double deta;         /* conformal time step, > 0 */
    double eta0;         /* conformal time of step 0, > 0 */
    double alpha;        /* damping coefficient of Eq. (2); PRS uses 3 */
    double beta;         /* scale-factor power of the force (0: PRS; 2: the exact equations) */
    double m;            /* era exponent d ln a / d ln eta (a ~ eta^m), >= 0 */
    double W0;           /* wall thickness parameter, > 0 (may be +inf) */
    double phi0;         /* vacuum value, > 0 */
    int32_t precision;   /* PRS_F32 (0, also a zero-initialised struct) or PRS_F64 */
    int32_t reserved;    /* must be 0 */
} prs_params;

#define PRS_F32 0   /* float32 fields: 16 B of HBM traffic per site-update */
#define PRS_F64 1   /* float64 fields: 32 B per site-update; tilings with vec 1 or 2 */

/* One diagnostic record (Eqs. 7-8) of the state (phi^n, phi_dot^{n-1/2}). */
typedef struct prs_stats {
    int64_t step;            /* n */
    double eta;              /* eta_n */
    uint64_t links;          /* forward links (i, i+e_d) whose sign changes */
    uint64_t links_dir[3];   /* the same per direction d */
    uint64_t wall_sites;     /* sites touching at least one such link */
    uint64_t nonfinite;      /* sites where phi or phi_dot is NaN or inf */
    double area_density;     /* rho = A/V, Eq. (7) */
    double gv2;              /* (gamma v)^2, Eq. (8); 0 when no wall site */
} prs_stats;

typedef struct prs_ctx prs_ctx;

/* ---- single run ------------------------------------------------------- */

/* Bytes of device workspace prs_init needs for these parameters (per-wave
 * diagnostic partial sums, the record buffer and a second phi_dot field for
 * multi-step passes); 0 if p is invalid. */
size_t prs_workspace_bytes(const prs_params* p);

/* Create a run context over caller-owned device buffers.
 *   phi_a, phi_b : two fields; phi_a holds phi^0 on entry, the evolution
 *                  ping-pongs between them (prs_get_state names the current)
 *   dphi         : phi_dot^{-1/2} on entry, updated in place
 *   workspace    : >= prs_workspace_bytes(p) bytes of device memory, 256-byte
 *                  aligned, owned by the caller and used only by this context
 * Validation (PRS_EINVAL): ndim, sides >= 1, dx, deta, eta0, W0, phi0 > 0,
 * m >= 0, alpha >= 0; the step must be stable for the linearised scheme,
 * deta * sqrt(4 D / dx^2 + 8 V0/phi0^2) < 2, and the first damping factor
 * must satisfy delta_0 = alpha m deta / (2 eta0) < 1; precision must be
 * PRS_F32 or PRS_F64 and reserved 0; beta finite.  With beta != 0 the force
 * changes with eta, and prs_step_n, prs_adjoint_forward and prs_batch_run
 * check the same stability bound with 8 V0 a^beta/phi0^2 at the largest
 * force of the call (PRS_EINVAL before any launch).  The persistent batch
 * modes take beta = 0 only.  The context starts at step 0. */
prs_status prs_init(const prs_params* p, void* phi_a, void* phi_b, void* dphi,
                    void* workspace, size_t ws_bytes, void* hip_stream, prs_ctx** out);

/* Number of diagnostic records prs_step_n(ctx at step n0, nsteps) produces:
 * the count of n in [n0, n0+nsteps) with n % diag_every == 0. */
int64_t prs_records_in(const prs_params* p, int64_t n0, int64_t nsteps);

/* Advance nsteps steps (Eqs. 3-6).  The Laplacian, kick and drift of a step
 * run fused in one kernel, and a launch advances up to steps_per_pass steps
 * at once (prs_set_time_blocking: default 2 in 2D, 1 in 3D; the autotuner
 * may choose up to 8 in 2D and 4 in 3D), never with a recorded state inside
 * a pass.  When series is non-NULL the diagnostics (Eqs. 7-8) of every state
 * n with n % diag_every == 0 are computed inside the pass that starts at n
 * (on its input state) and written to series[0 .. *n_written-1]; cap must be
 * at least prs_records_in(...), else PRS_EINVAL.  With series == NULL no
 * diagnostics are computed.  Splitting a call into two consecutive calls
 * gives bit-identical fields and records.  Synchronises the stream when
 * series is non-NULL or launch timing is on. */
prs_status prs_step_n(prs_ctx* ctx, int64_t nsteps, prs_stats* series, int64_t cap,
                      int64_t* n_written);

/* Diagnostics (Eqs. 7-8) of the current state; synchronises the stream.
 * The counts equal those of the record prs_step_n fuses for the same state;
 * the two FP64 sums are bitwise equal to it when that record came from a
 * single-step pass and equal up to summation order when it came from a
 * multi-step pass (which splits the lattice into different wave tiles). */
prs_status prs_wall_stats(prs_ctx* ctx, prs_stats* out);

/* Current state: device pointers of phi^n and phi_dot^{n-1/2}, n and eta_n.
 * Any output pointer may be NULL. */
prs_status prs_get_state(prs_ctx* ctx, void** phi, void** dphi, int64_t* step, double* eta);

/* Replace the state: copies the given device fields (any 16-byte aligned
 * device pointers; NULL keeps that field) into the context's buffers and sets
 * the step counter to `step` (>= 0). */
prs_status prs_set_state(prs_ctx* ctx, const void* phi, const void* dphi, int64_t step);

/* Choose the kernel tiling of this context (mainly for tests and the
 * autotuner).  vec: sites per lane along x (1, 2 or 4 in float32, 1 or 2 in
 * float64; must divide nx);
 * rows: planes per wave along the marching axis (y in 2D, z in 3D), 1..4096
 *   (the workspace holds the diagnostic partials of every tiling with rows
 *   >= 8, and of shorter ones only where the tiles still fit: PRS_EINVAL
 *   otherwise);
 * ty: in 3D, how a workgroup covers y: 1, 2 or 4 for one-wave workgroups
 * (single steps: 1, 2 or 4 rows per wave; multi-step passes: 4 rows per
 * wave, 8 with ty = 4), or 8, 16, 32, 64 for the LDS-staged multi-step
 * passes, whose workgroups stack waves along y and share their boundary rows
 * through LDS (8 waves of 2 or 4 rows for ty 8 or 16, 16 waves of 2 or 4
 * rows for ty 32 or 64; single steps on such a tiling use one row per
 * wave);
 * must be 1 in 2D.
 * Results are bit-identical for every tiling except the rounding order of the
 * two floating-point diagnostic sums. */
prs_status prs_set_tiling(prs_ctx* ctx, int32_t vec, int32_t rows, int32_t ty);
prs_status prs_get_tiling(prs_ctx* ctx, int32_t* vec, int32_t* rows, int32_t* ty);

/* Autotuner (Sec. IV: the kernels' work-group shapes were tuned for one
 * card, and another card needs them chosen again; here the choice is made
 * by timing on the card in use).  Times every supported tiling and steps per
 * pass for this lattice on the context's own state (saved into the caller's
 * workspace before and restored after each candidate) -- rows 8 to 128 in
 * powers of two and, for 2D multi-step passes (and the 2D reverse pass),
 * the row heights that make a pass's workgroup count a whole number of
 * rounds over the device's compute units where that count is small (up to
 * four workgroups per unit; eight for the reverse pass) -- applies the fastest
 * to the context and records it in the JSON file cache_path (created or
 * updated; NULL or "" for no cache).  A cached entry for the same GPU
 * architecture, dimension, lattice size and tiling set is applied without
 * timing (and without touching the workspace, which may then be NULL) unless
 * flags has PRS_TUNE_FORCE.  PRS_TUNE_BATCH restricts the candidates
 * (tilings and steps per pass) to those the persistent batch modes run
 * (prs_batch_run); the STREAMS batch modes take the ordinary choice.
 * PRS_TUNE_ADJOINT tunes the reverse sweep's tiling and steps per pass
 * instead, on scratch fields in the workspace.
 *   work, work_bytes : device scratch owned by the caller, 256-byte aligned,
 *                      at least prs_tune_workspace_bytes(ctx, flags) bytes
 *                      (PRS_ENOMEM otherwise); the library allocates nothing.
 *                      The adjoint tuner needs at least the size returned
 *                      with PRS_TUNE_MIN_WORKSPACE added to its flags and
 *                      fills what is beyond it with up to 32 distinct phi
 *                      fields, which the timed reverse steps read in
 *                      rotation as the backward does; with twelve or more,
 *                      the fused scheme's candidates are timed with the
 *                      recomputation running on a second stream beside the
 *                      reverse passes, each on half of the fields, as in
 *                      the backward.
 * *best_us (may be NULL) receives the time of one step with the chosen
 * tiling.  Synchronises. */
#define PRS_TUNE_FORCE 1
#define PRS_TUNE_BATCH 2
#define PRS_TUNE_ADJOINT 4   /* tune the reverse sweep's tiling and steps per pass instead */
#define PRS_TUNE_MIN_WORKSPACE 8   /* prs_tune_workspace_bytes: the least the tuner accepts */
size_t prs_tune_workspace_bytes(const prs_ctx* ctx, int32_t flags);
prs_status prs_autotune(prs_ctx* ctx, const char* cache_path, int32_t flags, void* work, size_t work_bytes,
                        double* best_us);

/* Launch timing, for measurement.  With on != 0, prs_step_n brackets every
 * run of consecutive launches of its pass kernel (the steps_per_pass-step
 * pass without diagnostics) with a pair of HIP events on the context's
 * stream, synchronises the stream before returning and adds the runs'
 * durations and launch counts to two totals.  prs_get_launch_timing reads
 * the totals (milliseconds and launches; either pointer may be NULL) and
 * clears them when reset != 0.  Off by default; timing adds two event
 * records per run of launches and changes no result. */
prs_status prs_set_launch_timing(prs_ctx* ctx, int32_t on);
prs_status prs_get_launch_timing(prs_ctx* ctx, double* total_ms, int64_t* launches, int32_t reset);

/* Plain device-to-device copy of `bytes` bytes (a multiple of 16) between
 * two 16-byte aligned, non-overlapping device buffers, enqueued on
 * hip_stream: the bandwidth reference the passes are measured against (a
 * pass moves its fields once, as a copy does).  PRS_EINVAL on a bad
 * argument, PRS_EDEVICE on a launch failure. */
prs_status prs_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Cached tiling for these parameters (no GPU work); PRS_ESTATE if absent. */
prs_status prs_tuned_tiling(const prs_params* p, const char* cache_path, int32_t flags, int32_t* vec,
                            int32_t* rows, int32_t* ty);

/* Temporal blocking: with steps_per_pass = T > 1, prs_step_n advances up to
 * T steps per pass over HBM -- a pass never has a recorded state inside it --
 * so each value is read about once per T steps.  T may be 2, 3, 4, 6 or 8 for
 * 2D lattices (default 2), and 2, 3 or 4 for 3D lattices (default 1); other
 * values give PRS_EINVAL.  A pass uses T steps only when the tiling has a
 * T-step kernel, and otherwise the longest length that has one:
 *   2D: ty = 1, any vec (in float64, T = 6 and 8 need vec 1).
 *   3D, one-wave tilings (ty 1, 2, 4): T = 2, 3 in float32 with vec 1, or
 *     vec 2 and ty 1 or 2; T = 2 in float64 with vec 1 and ty 1 or 2.
 *   3D, LDS tilings: T = 2, 3, 4; ty 8 and 16 with vec 1 (float32 and
 *     float64) or vec 2 (float32); ty 32 with vec 1 or 2 and ty 64 with vec 1,
 *     float32 only.
 * The autotuner picks T with the
 * tiling.  Results are bitwise those of single steps.  The second phi_dot
 * buffer this needs lives in the workspace; every prs_step_n call still ends
 * with phi_dot in the caller's dphi buffer.  Lattices whose rows (2D) reach
 * 2^28 sites or whose planes (3D) reach 2^31 bytes keep the setting but run
 * single-step passes. */
prs_status prs_set_time_blocking(prs_ctx* ctx, int32_t steps_per_pass);
prs_status prs_get_time_blocking(prs_ctx* ctx, int32_t* steps_per_pass);

/* How prs_step_n(ctx, nsteps, series != NULL iff with_records) would split
 * its steps: the number of multi-step passes and of single-step passes. */
prs_status prs_plan_passes(const prs_ctx* ctx, int64_t nsteps, int32_t with_records, int64_t* multi_passes,
                           int64_t* single_passes);

/* Tiling and steps per pass of the reverse sweep (adjoint), chosen
 * independently of the forward ones (same parameters and rules as
 * prs_set_tiling; PRS_TUNE_ADJOINT tunes both).  The forward-with-checkpoints
 * inside prs_adjoint_forward uses the forward tiling and steps per pass, and
 * so does the recomputation inside prs_adjoint_backward unless
 * prs_set_recompute_tiling sets its own (results depend on neither).
 * Multi-step reverse passes exist for 2D lattices with
 * T = 2, 4 and, in float32, 8 and tilings with vec 1 or 2, and for 3D
 * lattices with T = 2 on the one-wave tilings of the 3D multi-step passes
 * and, in float32, T = 3 with vec 1 and ty 1 or 2 (the LDS tilings, ty >= 8,
 * have no reverse pass and run single reverse steps); a pass runs the longest supported
 * length up to the setting, down to single reverse steps.  The default
 * tiling is the forward's at prs_init; the default steps per pass 4 in 2D,
 * 1 in 3D. */
prs_status prs_set_adjoint_tiling(prs_ctx* ctx, int32_t vec, int32_t rows, int32_t ty);
prs_status prs_get_adjoint_tiling(prs_ctx* ctx, int32_t* vec, int32_t* rows, int32_t* ty);
prs_status prs_set_adjoint_time_blocking(prs_ctx* ctx, int32_t steps_per_pass);
prs_status prs_get_adjoint_time_blocking(prs_ctx* ctx, int32_t* steps_per_pass);

/* How the backward gets the fields phi^n its reverse steps need (the
 * transposed Eqs. 3-6 read V''(phi^n) at every step n).
 *   PRS_ADJ_STORED: per segment of ckpt_every steps a recomputation from the
 *     checkpoint stores every step's field, and the reverse passes read them
 *     (4 B written and 4 B read per site and step in float32, besides the
 *     adjoint fields).
 *   PRS_ADJ_FUSED (2D lattices): the recomputation stores only the states
 *     (phi, phi_dot) at the starts of the reverse passes, steps_per_pass
 *     steps apart (2, 3 or 4: the adjoint steps per pass, capped at 4), and
 *     each reverse pass recomputes its fields in registers from its
 *     pass-start state (16 + 8 B per site per pass in float32); the reverse
 *     tiling then needs vec 1 or 2 (float64: vec 1) and ty 1.  A 3D lattice,
 *     or a setting without such a kernel, runs the stored scheme.
 * Gradient fields are bitwise equal in both schemes; dL/dW0 differs in
 * summation order.  Default: PRS_ADJ_FUSED for 2D, PRS_ADJ_STORED for 3D.
 * PRS_EINVAL for another value. */
#define PRS_ADJ_STORED 0
#define PRS_ADJ_FUSED 1
prs_status prs_set_adjoint_scheme(prs_ctx* ctx, int32_t scheme);
prs_status prs_get_adjoint_scheme(prs_ctx* ctx, int32_t* scheme);

/* Tiling and steps per pass (1 .. 8; the longest supported length up to it
 * is used, as in prs_set_time_blocking) of the recomputation inside
 * prs_adjoint_backward.  steps_per_pass = 0 makes it follow the forward's
 * setting again (the default; the other arguments are then ignored).  The
 * getter returns the setting in effect.  Results do not depend on it. */
prs_status prs_set_recompute_tiling(prs_ctx* ctx, int32_t vec, int32_t rows, int32_t ty, int32_t steps_per_pass);
prs_status prs_get_recompute_tiling(prs_ctx* ctx, int32_t* vec, int32_t* rows, int32_t* ty,
                                    int32_t* steps_per_pass);

/* One multi-step pass over a slab of a lattice cut along its last axis
 * (y in 2D, z in 3D): the per-device kernel of a lattice sharded along that
 * axis (each device holds a slab and exchanges halo rows or planes with its
 * neighbours between passes; this library does not communicate).  p
 * describes the slab: n[ndim-1] interior rows (2D) or planes (3D) of the
 * other extents, and the run's physics; n0 is the global step of the pass's
 * first step (it sets the coefficients).  phi_in/pi_in hold phi^{n0} and
 * phi_dot^{n0-1/2} on n[ndim-1] + 2*steps rows or planes: row or plane k is
 * global z0 - steps + k, so the first and last `steps` are the halo the
 * caller filled from the neighbouring slabs (for a single slab of a periodic
 * lattice: its periodic images).  phi_out/pi_out, with the same layout,
 * receive phi^{n0+steps} and phi_dot^{n0+steps-1/2} on the interior
 * steps .. steps+n[ndim-1]-1 only; the other axes stay periodic.  steps and
 * the tiling must have a multi-step kernel for this dimension (see
 * prs_set_time_blocking); the four buffers are distinct device buffers of
 * the precision p names, 16-byte aligned.  No diagnostics.  Enqueued on
 * hip_stream; results are bitwise those of the same steps on the whole
 * lattice. */
prs_status prs_slab_pass(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows, int32_t ty,
                         const void* phi_in, void* phi_out, const void* pi_in, void* pi_out, void* hip_stream);

/* The same pass with the wall diagnostics (Eqs. 7-8, as prs_wall_stats
 * defines them) of the slab's input state phi^{n0}, phi_dot^{n0-1/2} fused
 * in, over its interior sites: links point to rising coordinates, so a link
 * crossing the upper face into the halo counts in this slab and one crossing
 * the lower face in the slab below; wall sites see both halos.  The record
 * is that of the slab as a lattice of its own: links, links_dir, wall_sites
 * and nonfinite add up over the slabs of a lattice; area_density is
 * per interior site (weight by the slab's sites to combine) and gv2 per wall
 * site (weight by wall_sites).  scratch is a device buffer of at least
 * prs_slab_scratch_bytes(p, steps, vec, rows, ty) bytes, 16-byte aligned,
 * used by this call only.  Synchronises hip_stream and writes *record (host).
 * Errors as prs_slab_pass, plus PRS_EINVAL for a NULL record or scratch and
 * PRS_ENOMEM for a short scratch buffer. */
prs_status prs_slab_pass_stats(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows,
                               int32_t ty, const void* phi_in, void* phi_out, const void* pi_in, void* pi_out,
                               void* scratch, size_t scratch_bytes, prs_stats* record, void* hip_stream);

/* Scratch bytes prs_slab_pass_stats needs for this slab, pass length and
 * tiling; 0 when the parameters are invalid or no such pass kernel exists. */
size_t prs_slab_scratch_bytes(const prs_params* p, int32_t steps, int32_t vec, int32_t rows, int32_t ty);

/* prs_slab_pass_stats for callers that cannot allocate memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same pass and the same record, but the scratch is a statically allocated
 * device array of 4 MiB that the library holds on every device it runs on
 * until the process ends, and the record is written to the device pointer
 * record_dev (one prs_stats, 16-byte aligned) without synchronising
 * hip_stream.  Nothing is allocated and no host copy is made.
 *   Limits: prs_slab_scratch_bytes(p, steps, vec, rows, ty) must not
 *   exceed 4 MiB (about 104,000 wave tiles); a larger pass returns
 *   PRS_ENOMEM before any launch.  Other errors as prs_slab_pass_stats.
 *   Sharing: every call on one device uses that device's one array, so
 *   calls that overlap on one device (other streams, other threads) race and
 *   may return wrong records; calls in sequence are safe (each pass writes
 *   every scratch value it reads). */
prs_status prs_slab_pass_stats_static(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows,
                                      int32_t ty, const void* phi_in, void* phi_out, const void* pi_in,
                                      void* pi_out, prs_stats* record_dev, void* hip_stream);

/* Destroy a context (does not free caller-owned buffers).  NULL is a no-op. */
void prs_destroy(prs_ctx* ctx);

/* ---- adjoint (reverse-mode gradient through the evolution) ----------- */

/* Differentiable path: the loss of a run of nsteps steps from the context's
 * current state (phi^{n0}, phi_dot^{n0-1/2}) is
 *     L = sum_i V(phi_i^S)/V0 = sum_i (phi_i^2/phi0^2 - 1)^2,   S = n0 + nsteps,
 * and its gradient is taken with respect to phi^{n0}, phi_dot^{n0-1/2} and W0
 * (through V0 = pi^2/(2 W0^2) in the force of Eq. 4).  The reverse sweep is the
 * hand-derived transpose of Eqs. (3)-(6): with w the adjoint of
 * phi_dot^{n+1/2}, mu^n = mu^{n+1} + b_n (Lap w - V''(phi^n) w) and the
 * previous w = a_n w + deta mu^n (a_n = (1-delta_n)/(1+delta_n),
 * b_n = deta/(1+delta_n)).
 *
 * Memory: (phi, phi_dot) is checkpointed every ckpt_every steps; in reverse,
 * each segment is recomputed from its checkpoint and then swept backwards.
 * With two or more segments the recomputation of the next-older segment runs
 * on a second stream of the context while the current one is swept, into a
 * second segment buffer; results are the same as without the overlap.  All
 * of it lives in a caller-owned device workspace of
 * prs_adjoint_workspace_bytes(...) bytes (256-byte aligned), about
 * (2 nsteps/K + 2K + 4) fields (K + 4 with a single segment). */
size_t prs_adjoint_workspace_bytes(const prs_params* p, int64_t nsteps, int32_t ckpt_every);

/* Forward half: advances the context by nsteps (no diagnostics), storing the
 * checkpoints in `work`, and returns the loss (synchronises the stream).
 * nsteps >= 1, ckpt_every >= 1, else PRS_EINVAL; PRS_ENOMEM if work_bytes is
 * too small. */
prs_status prs_adjoint_forward(prs_ctx* ctx, int64_t nsteps, int32_t ckpt_every, void* work,
                               size_t work_bytes, double* loss);

/* Reverse half: must follow prs_adjoint_forward with the same workspace
 * (PRS_ESTATE otherwise; each forward allows one backward).  Writes
 * dL/dphi^{n0} to grad_phi0 and dL/dphi_dot^{n0-1/2} to grad_dphi0 (float32
 * device fields; either may be NULL) and dL/dW0 to *grad_W0 (may be NULL).
 * Leaves the context state at step S.  Synchronises the stream. */
prs_status prs_adjoint_backward(prs_ctx* ctx, void* work, size_t work_bytes, void* grad_phi0,
                                void* grad_dphi0, double* grad_W0);

/* Both halves in one call. */
prs_status prs_adjoint(prs_ctx* ctx, int64_t nsteps, int32_t ckpt_every, void* work,
                       size_t work_bytes, void* grad_phi0, void* grad_dphi0, double* grad_W0,
                       double* loss);

/* ---- batched ensemble -------------------------------------------------- */

/* An ensemble of independent realisations -- mixed 2D/3D lattices, sizes,
 * eras m, wall widths W0, time steps and step counts -- advanced together,
 * as needed for the large sets of production runs and the model calibration
 * the paper motivates (Secs. I and IV).  Each realisation follows exactly the
 * single-run method (same kernels per tile), so its fields and records are
 * bitwise those of the same realisation run alone with the same tiling. */
typedef struct prs_batch_item {
    prs_params p;        /* this realisation's parameters (diag_every: its cadence) */
    int64_t nsteps;      /* steps to run, >= 0 */
    uint64_t seed;       /* initial field seed (prs_fill_uniform) */
    int32_t init_from_seed;  /* 1: every run starts from the seeded field and
                                dphi = 0; 0: from the buffers' contents */
    int32_t reserved;
    void* phi_a;         /* caller-owned fields as in prs_init: phi_a holds phi^0; */
    void* phi_b;         /*   prs_batch_state names the buffer of the final phi */
    void* dphi;
} prs_batch_item;

typedef struct prs_batch prs_batch;

/* Execution modes.  Every mode runs each realisation's single-run pass plan
 * (its own tiling and steps per pass).  STREAMS launches the passes on one of
 * a few concurrent streams, realisations assigned longest-first to the least
 * loaded stream (the default); STREAMS_GRAPH captures that launch sequence
 * once in a hipGraph and replays it.  The PERSISTENT modes run the whole
 * ensemble inside one launch of a persistent kernel: the passes are cut into
 * work items (one to four wave tiles per wave of an 8-wave workgroup, or
 * workgroup tiles of a 3D LDS-staged pass), the realisations are dealt,
 * longest first, onto 16 sequences that each run their realisations' passes
 * one after another, the items are numbered round by round (round k: the
 * k-th pass of every sequence) and the workgroups take them from one
 * counter; an item waits only until its own realisation has finished the
 * previous pass (per-realisation counters, no grid barrier), and the
 * workgroup finishing a recorded pass reduces its record.  PER_STEP launches
 * the same kernel once per phase (phase p: pass p of every realisation).  They run float32 items with, in 2D, ty 1 and vec 1 or 2 (up to 8
 * steps per pass) or vec 4 (up to 4), and in 3D single steps with ty 1, or
 * vec 1 with ty 8 (up to 4 steps per pass) or ty 16 (up to 3). */
#define PRS_BATCH_PERSISTENT_GRAPH 0  /* one persistent launch, captured in a hipGraph */
#define PRS_BATCH_PERSISTENT 1        /* the same launch without the graph */
#define PRS_BATCH_PER_STEP 2          /* the same kernel, one launch per phase */
#define PRS_BATCH_STREAMS_GRAPH 3     /* concurrent streams, captured in a hipGraph */
#define PRS_BATCH_STREAMS 4           /* concurrent streams, launched directly (default) */

/* Device workspace (descriptors, coefficient and pass tables, the second
 * phi_dot field of 2D items, record partials and the records themselves); 0 if
 * any item is invalid. */
size_t prs_batch_workspace_bytes(const prs_batch_item* items, int32_t count);

/* Validates every item (as prs_init, PRS_EINVAL naming the item) and builds
 * the ensemble over caller-owned buffers and a 256-byte aligned workspace. */
prs_status prs_batch_create(const prs_batch_item* items, int32_t count, void* workspace,
                            size_t ws_bytes, void* hip_stream, prs_batch** out);

/* Records of item r occupy series[offsets[r] .. offsets[r+1]-1]: the states
 * n % diag_every == 0 for n < nsteps, then the final state n = nsteps.
 * offsets has count+1 entries. */
prs_status prs_batch_offsets(const prs_batch* b, int64_t* offsets);

/* Tiling of one item (as prs_set_tiling; see the execution modes for the
 * tilings the persistent modes run). */
prs_status prs_batch_set_tiling(prs_batch* b, int32_t item, int32_t vec, int32_t rows, int32_t ty);

/* Steps per pass of one item: 1, or a multi-step pass length as for
 * prs_set_time_blocking (2 is the default for 2D items, 1 for 3D items;
 * PRS_EUNSUPPORTED for rows or planes too long for multi-step passes; see
 * the execution modes for the lengths the persistent modes run).  The
 * second phi_dot field multi-step passes need lives in the workspace. */
prs_status prs_batch_set_time_blocking(prs_batch* b, int32_t item, int32_t steps_per_pass);

/* Current tiling and steps per pass of one item (any pointer may be NULL). */
prs_status prs_batch_get_tiling(const prs_batch* b, int32_t item, int32_t* vec, int32_t* rows, int32_t* ty,
                                int32_t* steps_per_pass);

/* Device pointers of item `item`'s final phi and phi_dot after prs_batch_run
 * (phi_dot is always the item's dphi buffer). */
prs_status prs_batch_state(const prs_batch* b, int32_t item, void** phi, void** dphi);
prs_status prs_batch_set_mode(prs_batch* b, int32_t mode);

/* Runs the whole ensemble (initial fields if init_from_seed, all steps, all
 * records) and synchronises the stream.  series may be NULL; otherwise cap
 * must hold offsets[count] records.  A wait of the persistent kernel lasts
 * at most 5 s (it only waits for items that running workgroups hold, so it
 * ends unless something has failed); past that the run stops with
 * PRS_EDEVICE instead of hanging.  PRS_EINVAL if the mode cannot run an
 * item's precision, tiling or steps per pass. */
prs_status prs_batch_run(prs_batch* b, prs_stats* series, int64_t cap);

/* Ensemble-level tuning (Sec. IV: settings re-chosen by measurement on the
 * card in use).  A realisation's own tuned setting is the fastest for it
 * alone; inside an ensemble the other realisations also fill the GPU, and in
 * the persistent modes taller tiles, which re-read fewer halo rows per
 * stored row, can win.  Starting from the current settings, for each group
 * of realisations that share a lattice and a setting (largest work first)
 * the tuner times the candidates -- the rows (2D) or planes (3D) of the
 * tiling doubled, up to 128, and for a 3D workgroup-stacked tiling (ty 8,
 * 16, 32, 64) each other such ty with the longest pass the mode runs for
 * it -- and keeps the fastest while the whole ensemble in the current mode
 * runs more than 2 % faster (each setting timed as the faster of two runs
 * after one untimed run); vec is kept, and settings the mode cannot run are
 * skipped.  Every item must have init_from_seed = 1 (PRS_EINVAL otherwise),
 * since the ensemble is run several times; the records of those runs are
 * discarded and the buffers hold the last run's final fields.  *best_ms (may
 * be NULL) receives the time of one run with the settings kept.
 * Synchronises; allocates nothing on the device. */
prs_status prs_batch_autotune(prs_batch* b, double* best_ms);

void prs_batch_destroy(prs_batch* b);

/* ---- initial conditions ---------------------------------------------- */

/* Fill count float32 values at device pointer phi with the seeded initial
 * field: site i gets (2k+1)/2^24 - 1 where k is the top 24 bits of the
 * SplitMix64 output for counter i+1 under `seed` (Steele, Lea & Flood 2014),
 * i.e. i.i.d. uniform on (-1, 1), exact in float32 and never 0.  The paper
 * generates its random initial conditions once in single precision and feeds
 * them to every run (Sec. III).  Asynchronous on the stream. */
prs_status prs_fill_uniform(void* phi, int64_t count, uint64_t seed, void* hip_stream);

/* The same values (exact float32 numbers) written as float64, for
 * PRS_F64 fields. */
prs_status prs_fill_uniform_f64(void* phi, int64_t count, uint64_t seed, void* hip_stream);

/* ---- scaling exponents (Eq. 9) --------------------------------------- */

/* Unweighted least-squares slopes mu of ln rho and nu of ln(gamma v) against
 * ln eta (Eq. 9), over the records with eta_min <= eta <= eta_max and
 * positive values (pass 0 / +inf for no bound).  Host-only. */
prs_status prs_fit_scaling(const prs_stats* series, int64_t count, double eta_min,
                           double eta_max, double* mu, double* nu);

/* ---- errors ----------------------------------------------------------- */

const char* prs_strerror(prs_status s);
const char* prs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PRS_H */
