/*
 * pa.h -- C ABI of the MI355X hot path for preconditioned adjoint data
 * assimilation of 2D turbulence (Ke, You & Wang, arXiv 2602.14016).
 *
 * What is computed
 *   Forward model: 2D incompressible Navier-Stokes (Sec. II.A, Eq. (1)), with
 *   the Kolmogorov body force f = (A sin(n_f y), 0) when forcing_amp != 0
 *   (Sec. III.E, Eq. (24)), integrated in vorticity form on the periodic box
 *   [0, 2pi)^2 on an N x N grid:
 *       d omega/dt = -(nu |k|^2 + mu) omega - P(u . grad omega) + P curl f
 *   with the 2/3-rule projector P (modes |kx|, |ky| <= Kc, k != 0, Kc the
 *   largest integer below N/3), u = d_y psi, v = -d_x psi, -Lap psi = omega,
 *   and the integrating-factor (Lawson) RK4 scheme with step dt.
 *   Cost (Sec. II.A, Eqs. (2)-(3)): J = 1/2 sum over observation steps and
 *   probes (x = i*stride, y = j*stride) of |u - m|^2, both components.
 *   Gradient: the exact discrete adjoint of that scheme (the paper's
 *   summation-by-parts adjoint, Sec. III; continuous form Eqs. (11)-(12)),
 *   returned as dJ/d omega0 in the grid-Euclidean inner product.
 *   Preconditioner: Fourier multiplier (m(k)^2 W(|k|))^p with W one of the
 *   kernels of Sec. III.B (plus exp(-sigma|k|)), m^2 = |k|^2 (velocity
 *   metric), 1 (vorticity metric) or |k|^4 (streamfunction metric: the
 *   control variables u0, omega0, psi0 of Sec. III.A); latent control s = G^(-1/2) omega0 and
 *   latent gradient G^(1/2) dJ/domega0 (Sec. II.B-C, Eqs. (13)-(19)).
 *   Optimiser: L-BFGS or steepest descent in the latent control (Sec. II.C).
 *
 * Conventions
 *   - Every function returns pa_status: PA_OK (0) or a negative error code.
 *     Nothing throws or aborts across the ABI; pa_last_error() returns a
 *     message for the calling thread's most recent failure.
 *   - Arguments are validated before any device call; on a validation error
 *     nothing is enqueued and no output is touched.  Every pointer documented
 *     as "device" must be device (or managed) memory; host memory is refused
 *     with PA_EINVAL (pa_is_device_memory).
 *   - "device" pointers are HIP device memory owned by the caller (e.g. torch
 *     tensors); "host" pointers are ordinary host memory.  The library owns only
 *     the opaque context (plans and small constant tables it allocates in
 *     pa_create and frees in pa_destroy).
 *   - Work is enqueued asynchronously on the context's HIP stream (set at
 *     creation or with pa_set_stream).  Functions that return host values
 *     synchronise that stream; the others do not.
 *   - Physical fields are FP64 arrays [B][N][N], row-major, f[b][j][i] at
 *     (x_i, y_j) = (2 pi i / N, 2 pi j / N).  All arithmetic is FP64.
 *   - Workspaces and checkpoint buffers are opaque device memory of the size
 *     reported by the *_bytes queries, 256-byte aligned, caller-owned.  Calls
 *     that share a workspace on one stream are serialised by the stream;
 *     concurrent calls on different streams need different workspaces.
 *   - A context is used by one host thread at a time: its settings (tiles,
 *     Sobolev weight, snapshot budget), its cached checkpoint schedule and
 *     its launch timer are not locked.  Different contexts may be used from
 *     different threads at once.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pa_status;

#define PA_OK            0
#define PA_EINVAL       (-1)  /* bad argument (size, pointer, parameter)      */
#define PA_ENOMEM       (-2)  /* workspace too small / device allocation failed */
#define PA_EDEVICE      (-3)  /* HIP runtime error or no device                */
/* Reserved; no call of this version returns them.  Per-member outcomes of an
 * assimilation (a line-search failure, a non-finite cost) are reported in
 * iters_done and J_hist, and the call itself returns PA_OK. */
#define PA_ENONFINITE   (-4)  /* non-finite value met                          */
#define PA_ELINESEARCH  (-5)  /* Armijo line search failed (step collapse)     */
#define PA_EUNSUPPORTED (-6)  /* valid request this version does not support   */

typedef struct pa_ctx pa_ctx;

/* Physical parameters (Sec. II.A Eq. (1), Sec. III.E Eq. (24)).
 * nu >= 0 viscosity, mu >= 0 linear drag, dt > 0 time step,
 * forcing_amp = A and forcing_k = n_f of f = (A sin(n_f y), 0); A = 0: decaying. */
typedef struct pa_physics {
    double  nu;
    double  mu;
    double  dt;
    double  forcing_amp;
    int32_t forcing_k;
    int32_t reserved;          /* must be 0 */
} pa_physics;

/* Observation set (Sec. II.A Eq. (3)).  Probes at (x, y) = (i*stride, j*stride)
 * grid points, i, j in [0, M), M = N / stride; stride must divide N.
 * steps: host array of n_times strictly increasing step indices in
 * [0, n_steps].  values: device array [B][n_times][2][M][M] (component 0 = u,
 * 1 = v), or NULL when only model observations are wanted.  Caller-owned. */
typedef struct pa_obs {
    int32_t        stride;
    int32_t        n_times;
    const int32_t* steps;
    const double*  values;
} pa_obs;

/* Weighting kernel W(|k|) and control metric (Sec. II.B-C; Sec. III.B).
 * kind 0: identity W = 1
 *      1: exponential W = exp(-param |k|)
 *      2: fractional  W = |k|^(-2 param)
 *      3: heat kernel W = exp(-param |k|^2)    (param = nu*beta of the paper)
 * metric 0: velocity (m^2 = |k|^2), 1: vorticity (m^2 = 1), 2: streamfunction
 * (m^2 = |k|^4): with W = 1 the latent control's Euclidean norm is that of
 * u0, omega0 or psi0 (Sec. III.A).  W(0) = 1. */
typedef struct pa_kernel {
    int32_t kind;
    int32_t metric;
    double  param;
} pa_kernel;

/* Largest batch of one context: members index the second launch-grid
 * dimension, which holds at most 65535 workgroups. */
#define PA_MAX_MEMBERS 65535

/* Create a context for B fields of size N x N (N a power of two in
 * [8, 1024], 1 <= B <= PA_MAX_MEMBERS) with the given physics, enqueueing on hip_stream
 * (hipStream_t, NULL = default stream).  Allocates small constant tables on
 * the current device.  Errors: PA_EINVAL (bad sizes/parameters, NULL out),
 * PA_EDEVICE (no device / HIP failure), PA_ENOMEM. */
pa_status pa_create(const pa_physics* phys, int32_t N, int32_t B,
                    void* hip_stream, pa_ctx** out);

/* Destroy a context (NULL is accepted).  Synchronises its stream first. */
pa_status pa_destroy(pa_ctx* ctx);

/* Change the stream later calls enqueue on. */
pa_status pa_set_stream(pa_ctx* ctx, void* hip_stream);

/* Message for the calling thread's most recent error ("" if none). */
const char* pa_last_error(void);

/* Query: N, B, Kc (band limit) of a context. */
pa_status pa_get_shape(const pa_ctx* ctx, int32_t* N, int32_t* B, int32_t* Kc);

/* Workspace bytes for a gradient over n_steps with checkpoints every
 * ckpt_every steps (1 <= ckpt_every), n_obs_times observation times, and an
 * L-BFGS memory lbfgs_m (0 when not assimilating).  Any call documented as
 * taking "a workspace" accepts one of at least this size for its arguments;
 * pa_precondition and pa_init_field need pa_workspace_bytes(ctx,0,1,0,0).
 * The size depends on the context's snapshot budget (pa_set_checkpoint_slots)
 * at the time of the query, which must not grow before the workspace is used. */
pa_status pa_workspace_bytes(const pa_ctx* ctx, int32_t n_steps, int32_t ckpt_every,
                             int32_t n_obs_times, int32_t lbfgs_m, size_t* bytes);

/* Bytes of the checkpoint buffer written by pa_forward (ceil(n_steps /
 * ckpt_every) + 1 spectral states per member). */
pa_status pa_checkpoint_bytes(const pa_ctx* ctx, int32_t n_steps, int32_t ckpt_every,
                              size_t* bytes);

/* Seeded initial vorticity fields (Sec. III: prescribed spectrum, random
 * phases, normalised energy).  seeds: host [B].  kind 0: random phase with
 * |omega_hat| = sqrt(|k| E(|k|)), E(k) = k^4 exp(-2 (k/k0)^2), kinetic
 * energy 1/2 <|u|^2> = target; kind 1: same spectrum with complex Gaussian
 * coefficients; kind 2: white noise on the de-aliased band with RMS(omega) =
 * target.  Random numbers: SplitMix64 keyed by (seed, wavevector, stream), so
 * a seed gives the same low modes at every N.  omega_out: device [B][N][N]. */
pa_status pa_init_field(pa_ctx* ctx, const uint64_t* seeds, int32_t kind, double k0,
                        double target, double* omega_out, void* workspace,
                        size_t workspace_bytes);

/* Forward solve over n_steps from omega0 (device [B][N][N]; P is applied to
 * it first).  Optional outputs (NULL to skip):
 *   omega_T  device [B][N][N]   final vorticity
 *   obs      observation set; with obs->values the cost J is computed
 *   J_out    device [B]         cost per member (needs obs->values)
 *   obs_out  device [B][n_times][2][M][M]  model observations M u
 *   ckpt     device, pa_checkpoint_bytes, 16-byte aligned (PA_EINVAL
 *            otherwise): spectral states every ckpt_every steps, the input
 *            of pa_adjoint_from_checkpoints. */
pa_status pa_forward(pa_ctx* ctx, const double* omega0, int32_t n_steps,
                     const pa_obs* obs, double* J_out, double* obs_out, double* omega_T,
                     int32_t ckpt_every, void* ckpt, void* workspace, size_t workspace_bytes);

/* Gradient dJ/d omega0 (device [B][N][N]) and J (device [B], may be NULL)
 * by a checkpointed forward sweep, segment-wise recomputation and the
 * discrete adjoint sweep.  obs->values is required. */
pa_status pa_adjoint_gradient(pa_ctx* ctx, const double* omega0, int32_t n_steps,
                              const pa_obs* obs, double* J_out, double* grad_out,
                              int32_t ckpt_every, void* workspace, size_t workspace_bytes);

/* Scratch that pa_adjoint_gradient_noalloc uses in place of a workspace:
 * 128 MiB of device memory per device the library runs on, reserved when the
 * library's code is loaded there and held until the process ends. */
#define PA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * gradient of pa_adjoint_gradient, bit for bit, with its workspace carved
 * from a library-owned device array of PA_NOALLOC_SCRATCH_BYTES instead of a
 * caller's buffer.  The caller passes inputs and outputs only (omega0, obs,
 * J_out, grad_out as in pa_adjoint_gradient).  No device memory is allocated
 * or freed, nor host memory on success (launch timing by pa_profile_start
 * creates its events).  The internal checkpoints keep one state per segment
 * boundary: PA_EINVAL if a snapshot budget (pa_set_checkpoint_slots) would
 * make a binomial schedule, and PA_EINVAL, with the size needed, when
 * pa_workspace_bytes(ctx, n_steps, ckpt_every, obs->n_times, 0) exceeds
 * PA_NOALLOC_SCRATCH_BYTES (lower ckpt_every or use pa_adjoint_gradient).
 * Every call on one device shares that device's array and leaves its
 * contents behind; calls that overlap in time on one device (other streams,
 * other threads, other contexts) race on it and must be serialised by the
 * caller.  Contexts on different devices use different copies. */
pa_status pa_adjoint_gradient_noalloc(pa_ctx* ctx, const double* omega0, int32_t n_steps,
                                      const pa_obs* obs, double* J_out, double* grad_out,
                                      int32_t ckpt_every);

/* Same gradient from the checkpoints a previous pa_forward wrote (same
 * n_steps, ckpt_every, obs steps; ckpt 16-byte aligned).  scale: device [B]
 * or NULL; the gradient of member b is multiplied by scale[b] (the autograd
 * backward's grad_output). */
pa_status pa_adjoint_from_checkpoints(pa_ctx* ctx, const void* ckpt, int32_t n_steps,
                                      const pa_obs* obs, const double* scale,
                                      double* grad_out, int32_t ckpt_every,
                                      void* workspace, size_t workspace_bytes);

/* out = F^-1[(m^2 W)^power 1_S F in] (device [B][N][N] each; in == out is
 * allowed).  power = -1/2 maps omega0 to the latent control, +1/2 maps back
 * and turns dJ/domega0 into the latent gradient, 1 gives the filtered
 * gradient G dJ/domega0 (Eq. (17)). */
pa_status pa_precondition(pa_ctx* ctx, const pa_kernel* kernel, double power,
                          const double* in, double* out, void* workspace,
                          size_t workspace_bytes);

/* Preconditioned 4D-Var (Sec. II.C): minimise J over the latent control
 * s = precondition(omega, -1/2) from the first guess omega_inout (device
 * [B][N][N]; overwritten with precondition(s_final, +1/2)).  method 0:
 * L-BFGS with memory lbfgs_m (two-loop recursion, H0 = (s.y / y.y) I);
 * 1: steepest descent.  Trial step J/|g|^2 on the first iteration or after a
 * memory reset, else 1; backtracking Armijo (c1 = 1e-4, halving, 30 trials).
 * J_hist: host [B][max_iter + 1], the cost after each accepted iteration
 * (unused entries NaN).  iters_done: host [B], iterations completed, negated
 * minus one (-(k+1)) if member b stopped on a line-search failure after k
 * iterations (a non-finite cost, e.g. from a NaN observation, fails every
 * trial step and ends there too).  Members run in one batch; a failure stops
 * only that member.
 * Synchronises the stream. */
pa_status pa_assimilate(pa_ctx* ctx, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                        const pa_kernel* kernel, int32_t method, int32_t max_iter,
                        int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                        int32_t* iters_done, void* workspace, size_t workspace_bytes);

/* pa_assimilate with one kernel per member (kernels: host array of B): a
 * sweep over preconditioners (kernel families and parameters) as one batched
 * solve, e.g. the fractional exponent or the heat-kernel parameter across
 * members (Sec. III.B-C).  Member b follows exactly the iterations
 * pa_assimilate would run for it alone with kernels[b]. */
pa_status pa_assimilate_kernels(pa_ctx* ctx, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                const pa_kernel* kernels, int32_t method, int32_t max_iter,
                                int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                                int32_t* iters_done, void* workspace, size_t workspace_bytes);

/* pa_assimilate_kernels with one observation set per member: the requests
 * of a serving queue that share a grid and physics but differ in horizon,
 * probe stride, observation times and kernel, as one batched solve
 * (Sec. II.A Eqs. (2)-(3) per member; Sec. II.C).  obs: host array of B
 * sets, each with its own stride, n_times >= 1 increasing steps and values
 * (device [1][n_times][2][M_b][M_b] of that member alone, M_b = N / stride_b);
 * kernels: host array of B.  A member's horizon is its last observation
 * step; n_steps must be the latest of them.  Member b advances only through
 * its own horizon (the steps past it are not computed for it), and its cost,
 * gradients, iterates, J_hist row and iteration count are those of
 * pa_assimilate_kernels run for it alone with its own horizon, bit for bit.
 * Members ordered by decreasing horizon share every launch of a step; the
 * order does not change results.  Workspace: pa_workspace_bytes(ctx,
 * n_steps, ckpt_every, largest n_times, lbfgs_m).  The snapshot budget must
 * be 0 (one checkpoint per segment boundary).  PA_EINVAL for a member
 * without observations or n_steps other than the latest horizon.
 * Synchronises the stream. */
pa_status pa_assimilate_members(pa_ctx* ctx, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                const pa_kernel* kernels, int32_t method, int32_t max_iter,
                                int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                                int32_t* iters_done, void* workspace, size_t workspace_bytes);

/* Cancellation of running 4D-Var members: flags is host memory [B] (or
 * NULL to switch it off) that pa_assimilate* read, never write, at every
 * iteration boundary; another thread may set an entry non-zero at any time.
 * A member whose flag is set stops before its next iteration: its field, cost
 * history and iteration count (positive) are those of its last completed
 * iteration, and the other members run on unchanged.  With a state_out
 * (pa_assimilate_ex) the cancelled member is recorded as paused, so a resume
 * continues it; when the whole batch is cancelled at one boundary, the
 * resumed run is bit for bit the uninterrupted one (a member paused while
 * others go on keeps fewer stored pairs).  The pointer stays in use until it
 * is replaced or cleared. */
pa_status pa_set_cancel_flags(pa_ctx* ctx, const int32_t* flags);

/* Bytes of an optimiser state of this context for memory lbfgs_m (per_member:
 * one kernel per member, as in pa_assimilate_kernels): a header, the O(B m)
 * scalars of the batched line searches and pair ring, the latent iterate and
 * gradient, and the m stored pairs (about (2 + 2m) B N^2 doubles). */
pa_status pa_assimilate_state_bytes(const pa_ctx* ctx, int32_t lbfgs_m, int32_t per_member, size_t* bytes);

/* pa_assimilate (per_member = 0, kernels: one kernel) or pa_assimilate_kernels
 * (per_member = 1, kernels: B) that can stop and resume (the optimiser
 * restart of an interrupted 4D-Var).  state_out (device, may be NULL): after
 * the last iteration the gradient at the final iterate is taken and its pair
 * stored, as a longer run would, and the whole optimiser state is written
 * there.  state_in (device, may be NULL, may equal state_out): the run
 * continues from that state instead of from omega_inout (which is then
 * output only), so k iterations written out and j more resumed give the
 * iterates, costs and final field of one run of k + j iterations bit for bit.
 * J_hist[b][0] is then the cost at the resumed point and iters_done counts
 * from the first run.  Each state is state_bytes >= pa_assimilate_state_bytes
 * bytes, 256-byte aligned; a state is a plain byte image (it can be copied to
 * host memory or a file and back).  PA_EINVAL if state_in was written for
 * other sizes, method, memory, window length, observation times or stride,
 * or other kernels.  The caller keeps the observations and physics the same. */
pa_status pa_assimilate_ex(pa_ctx* ctx, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                           const pa_kernel* kernels, int32_t per_member, int32_t method,
                           int32_t max_iter, int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                           int32_t* iters_done, const void* state_in, void* state_out,
                           size_t state_bytes, void* workspace, size_t workspace_bytes);

/* Running sums of an ensemble of impulse responses, accumulated by
 * pa_adjoint_impulse over any number of calls (batches of members), for the
 * ensemble statistics of Sec. IV.  The caller allocates the device buffers
 * (sizes from pa_ensemble_acc_bytes), zeroes them and sets count = 0 before
 * the first batch; each call adds its B members, one at a time in member
 * order, and adds B to count, so any split of an ensemble into batches gives
 * bitwise the same sums.
 *   lambda_sum  device, complex [n_steps + 1][2Kc + 1][KXP] (the compact
 *               spectral layout: kx = 0..Kc of each ky row, padded to KXP =
 *               8 * ceil((Kc + 1) / 8); padding is never written): sum over
 *               members of the adjoint state at each backward step
 *   energy_sum  device [n_steps + 1]: sum over members of the total adjoint
 *               energy sum_k 1/2 |k|^2 |lambda_hat|^2 / N^4
 *   shell_sum   device [n_steps + 1][n_shells]: sum over members of the
 *               shell energies (the n_shells of the accumulating calls) */
typedef struct pa_ensemble_acc {
    void* lambda_sum;
    double* energy_sum;
    double* shell_sum;
    int64_t count;
} pa_ensemble_acc;

pa_status pa_ensemble_acc_bytes(const pa_ctx* ctx, int32_t n_steps, int32_t n_shells, size_t* lambda_bytes,
                                size_t* energy_bytes, size_t* shell_bytes);

/* Adjoint impulse response (Sec. IV): forward n_steps from omega0, then the
 * adjoint from a unit u-impulse at grid point (ix, iy) at the final step.
 * shells_out: device [B][n_steps + 1][n_shells], row r = backward step r
 * (tau = r dt, row 0 the terminal field), entry k-1 = sum over
 * k <= |k| < k+1 of 1/2 |k|^2 |lambda_hat|^2 / N^4 (Eq. (20) with unit shell
 * width).  field_out: device [B][N][N] or NULL, P lambda at step 0.
 * acc: NULL, or ensemble sums to add this batch to (see pa_ensemble_acc;
 * its shell_sum has n_shells columns). */
pa_status pa_adjoint_impulse(pa_ctx* ctx, const double* omega0, int32_t n_steps,
                             int32_t ix, int32_t iy, int32_t n_shells, double* shells_out,
                             double* field_out, pa_ensemble_acc* acc, int32_t ckpt_every,
                             void* workspace, size_t workspace_bytes);

/* Ensemble statistics from accumulated sums (Sec. IV), per backward step
 * r < rows (rows <= n_steps + 1 of the accumulation), all device outputs:
 *   mean_energy      [rows][n_shells]  mean over members of the shell energy
 *   energy_of_mean   [rows][n_shells]  shell energy of the ensemble-mean adjoint
 *   total_mean       [rows]            mean over members of the total adjoint energy
 *   total_of_mean    [rows]            total energy of the ensemble-mean adjoint
 *   snr              [rows]            total_of_mean / total_mean
 * n_shells must equal the accumulating calls' n_shells.  PA_EINVAL if
 * acc->count < 1 or a pointer is NULL. */
pa_status pa_ensemble_stats(pa_ctx* ctx, const pa_ensemble_acc* acc, int32_t rows, int32_t n_shells,
                            double* mean_energy, double* energy_of_mean, double* total_mean,
                            double* total_of_mean, double* snr);

/* First guess from the probe velocities at t = 0 (the paper's "initial
 * interpolated state", Sec. III.A): spectral interpolation of the M x M probe
 * grid (M = N / stride) -- the coarse Nyquist row and column are dropped --
 * then omega_hat = i kx v_hat - i ky u_hat on the de-aliased band.
 * probes: device [B][2][M][M] (u then v); omega_out: device [B][N][N];
 * workspace: at least pa_workspace_bytes(ctx, 0, 1, 0, 0). */
pa_status pa_first_guess(pa_ctx* ctx, int32_t stride, const double* probes, double* omega_out,
                         void* workspace, size_t workspace_bytes);

/* Ensemble statistics of pa_adjoint_impulse output (Sec. IV): shells is
 * device [B][rows][n_shells]; mean_out (device [rows][n_shells], may be NULL)
 * receives the member mean, rate_out (device [n_shells]) the least-squares
 * slope of ln(mean) against backward time tau = row * dt over
 * [tau_min, tau_max] (NaN where undefined). */
pa_status pa_shell_growth(pa_ctx* ctx, const double* shells, int32_t rows, int32_t n_shells,
                          double tau_min, double tau_max, double* mean_out, double* rate_out);

/* FFT tile choice of a context (the autotuner's knobs), per pass: the forward
 * row passes (right-hand side products, observation, transforms of physical
 * fields), the adjoint row passes (adjoint products, source rows) and the
 * column pass.  variant = register plan of the 1D transforms (0: more
 * elements per thread, 1: more threads per transform, 2: four elements per
 * thread where the length allows; 3, row passes only: the plan of variant 2
 * run by persistent wavefronts that prefetch their next rows from HBM into
 * LDS, bitwise equal to variant 2); teams = rows per row-pass workgroup (1,
 * 2, 4 or 8, capped at 256 threads and 64 KiB of LDS per workgroup; with
 * variant 3, wavefronts per workgroup, capped at 4); col_block =
 * kx columns per column-pass workgroup (1, 2, 4 or 8, with col_block times
 * threads per transform <= 512 and LDS within the device's per-workgroup
 * limit, 160 KiB on gfx950; the default stays within 64 KiB); col_split = workgroups
 * per column that share out the column's output transforms, each recomputing
 * the input transform (0: chosen per launch, 2 or 4 shares where the launch
 * has fewer than two wavefronts per SIMD without them; 1, 2 or 4: fixed,
 * capped at the launch's output count).  Results do not depend on the choice
 * beyond rounding of the transforms, and not at all on col_split. */
typedef struct pa_tiles {
    int32_t row_variant, row_teams;
    int32_t adj_variant, adj_teams;
    int32_t col_variant, col_block;
    int32_t col_split;
} pa_tiles;

/* Sets the tiles; a negative field keeps its current value (a kept col_block
 * is reduced if the column variant needs it).  PA_EINVAL for values outside
 * the sets above or an explicit col_block that does not fit; nothing changes
 * then. */
pa_status pa_set_tiles(pa_ctx* ctx, const pa_tiles* tiles);

/* Sobolev regularisation of the cost (Eq. (4)): J += (lambda/2) int |grad
 * u0|^2 dOmega = (lambda/2) int omega0^2 dOmega (periodic, divergence-free),
 * evaluated exactly on the grid for P omega0 as (lambda/2) (2 pi/N)^2
 * sum_ij (P omega0)^2; the gradient gains lambda (2 pi/N)^2 P omega0.
 * Applies to every cost and cost gradient of this context (pa_forward's J,
 * pa_adjoint_gradient, pa_adjoint_from_checkpoints, pa_assimilate*), not to
 * impulse responses.  lambda = 0 (the default) switches it off; PA_EINVAL for
 * a negative or non-finite lambda. */
pa_status pa_set_sobolev(pa_ctx* ctx, double lambda);

/* Most segments a binomial schedule covers: the schedule is a host list of
 * at most about two actions per segment. */
#define PA_MAX_SCHEDULE_SEGMENTS (1 << 22)

/* Snapshot budget of the checkpoints kept inside the workspace by
 * pa_adjoint_gradient, pa_adjoint_impulse and pa_assimilate* (the adjoint's
 * recomputation, Sec. I and Sec. II.A).  The horizon splits into L =
 * ceil(n_steps / ckpt_every) segments; each segment is recomputed once with
 * all its stage fields kept before the adjoint runs through it.  slots = 0
 * (the default), or slots > L: the state at every segment boundary is kept
 * (L + 1 spectral states per member) and the forward runs once more in all.
 * 1 <= slots <= L: only `slots` spectral states per member are kept (the
 * first holds the initial state) and the segments are reversed by the
 * binomial schedule of Griewank & Walther, which re-advances the fewest
 * segments for that budget (pa_checkpoint_advances).  Results are the same
 * either way, bit for bit: only the schedule changes.  pa_forward and
 * pa_adjoint_from_checkpoints keep the caller's one-per-boundary layout.
 * PA_EINVAL for slots < 0, and from a solve whose binomial schedule would
 * cover more than PA_MAX_SCHEDULE_SEGMENTS segments. */
pa_status pa_set_checkpoint_slots(pa_ctx* ctx, int32_t slots);

/* Current snapshot budget of the context. */
pa_status pa_get_checkpoint_slots(const pa_ctx* ctx, int32_t* slots);

/* Host only (no device, no context).  Segment advances (forward segment
 * runs without stored fields, the first forward sweep included) of the
 * schedule that reverses n_segments segments with `slots` snapshot slots:
 * t L - C(s + t + 1, t - 1) for s = slots - 1 free slots, where t is the
 * least integer with C(s + 1 + t, t) >= L; L (L - 1) / 2 for one slot and
 * L - 1 for slots >= L.  Each segment is also run once with its fields
 * kept.  PA_EINVAL unless n_segments >= 1 and slots >= 1. */
pa_status pa_checkpoint_advances(int32_t n_segments, int32_t slots, int64_t* advances);

/* Host only.  The schedule itself: *n_actions actions, and if actions is not
 * NULL (host, at least 5 * capacity int32), each as (kind, a, b, src, dst):
 *   kind 0, advance: run segments a .. b-1 from the state in slot src (-1:
 *           the state the previous action left), keep the state of boundary
 *           b in slot dst (-1: none);
 *   kind 1, reverse: run segment a keeping its stage fields, from slot src
 *           (-1: the state the previous advance left), then the adjoint
 *           steps through it.
 * Slot 0 holds boundary 0 throughout.  The actions before the first reverse
 * form the forward sweep.  PA_EINVAL if capacity < *n_actions (n_actions is
 * still set), for sizes as in pa_checkpoint_advances, or for n_segments >
 * PA_MAX_SCHEDULE_SEGMENTS. */
pa_status pa_checkpoint_schedule(int32_t n_segments, int32_t slots, int32_t* actions, int64_t capacity,
                                 int64_t* n_actions);

/* Whether ptr is memory the kernels may dereference (device or managed
 * memory), the check every call makes on its device arguments before it
 * enqueues anything (PA_EINVAL "... is not device memory" otherwise).
 * *is_device = 0 for NULL and host memory.  Needs a device. */
pa_status pa_is_device_memory(const void* ptr, int32_t* is_device);

/* Current tiles of the context. */
pa_status pa_get_tiles(const pa_ctx* ctx, pa_tiles* tiles);

/* Launch timing for measurement: until pa_profile_stop, every sample_every-th
 * launch of one kernel class is bracketed by HIP events recorded on the
 * context stream (the stream the kernel runs on).  kernel_class 0: row pass
 * of the right-hand side; 1: column pass of the forward RK4 stages; 2: row
 * pass of the adjoint products; 3: column pass of the adjoint stages.
 * pa_profile_stop synchronises the stream and returns the number of timed
 * launches, the number of launches of that class seen, and the summed event
 * time in milliseconds. */
pa_status pa_profile_start(pa_ctx* ctx, int32_t kernel_class, int32_t sample_every);
pa_status pa_profile_stop(pa_ctx* ctx, int64_t* timed_launches, int64_t* seen_launches,
                          double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
