// kernels.hpp -- data layout, kernel argument blocks and launcher declarations.
//
// Layout in HBM (per context: N grid, B members, Kc = largest integer < N/3):
//   physical field   double [B][N][N]                f[b][y][x]
//   spectral state   cd     [B][KY][KXP]  ("compact") only the de-aliased band:
//                    row r <-> ky = r (r <= Kc) or r - KY (r > Kc), KY = 2 Kc + 1,
//                    column kx = 0..Kc, padded to KXP (multiple of 8) columns.
//                    Unnormalised DFT coefficients of the real field (the
//                    conjugate half kx < 0 is implied).
//   y-field          cd     [B][N][KXP]   ("Y")  a field after the x-direction
//                    real transform, kx = 0..Kc kept: the hand-off between the
//                    row pass (physical space, x contiguous) and the column
//                    pass (spectral space, transform along y).
//   packed y-fields  the fields that row passes read in pairs (A, B) -- the
//                    RK stage fields (u, w_x), (v, w_y) and the adjoint's
//                    (Lam_x, Lam_y) -- are stored as P = A + i B and
//                    Q = A - i B (each [B][N][KXP]): entry e of the row's full
//                    complex signal A + i B is P[e] for e <= Kc and conj(Q[N-e])
//                    for e >= N - Kc, one 16-byte load either way.
// Every 2D transform is a row pass + a column pass over Y; pointwise spectral
// work (projection, Poisson inversion, velocity, derivatives, Lawson RK4
// combine, adjoint transposes) is fused into the column pass, products of
// fields into the row pass.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "fft.hpp"

namespace pa {

struct Dims {
    int N, B, K, KX, KXP, KY;
    int var, tpb;    // forward row passes: FFT plan variant (0..3; 3 = pipelined), rows (waves) per workgroup
    int avar, atpb;  // adjoint row passes: FFT plan variant (0..3), rows (waves) per workgroup
    int cvar, cb;    // column pass: FFT plan variant, kx columns per workgroup
    int csplit;      // column pass: workgroups per column sharing its outputs (0: chosen per launch)
    int cus;         // compute units of the device (persistent grids)
    int lds_max;     // bytes of LDS a workgroup may use on the device (column blocks beyond 64 KiB)
};

// Column-pass outputs: the field itself, or one half of a packed pair
// (P = A + i B, Q = A - i B) with (A, B) = (u, w_x), (v, w_y) or (Lam_x, Lam_y).
enum FieldKind : int { F_OMEGA = 0, F_UP = 1, F_UQ = 2, F_VP = 3, F_VQ = 4, F_LP = 5, F_LQ = 6 };

// Multiplier applied to an adjoint column input after its y-transform.  The
// adjoint row pass stores its two products (G1, G2) unsplit, as P = Z and
// Q = conj Z(-k) of Z = F_x(G1 + i G2), so G1 = (P + Q)/2 and G2 = (P - Q)/(2i),
// and the column pass's 1/|k|^2 G1 + G2 becomes P (1/|k|^2 - i)/2 + Q (1/|k|^2 + i)/2.
enum InMul : int { IN_PAIRP = 0, IN_PAIRQ = 1, IN_IKY_INVK2 = 2, IN_MIKX_INVK2 = 3 };

enum ColMode : int {
    COL_INIT = 0,     // Y -> P omega0 -> state (+checkpoint) -> derived fields
    COL_A = 1, COL_B = 2, COL_C = 3, COL_D = 4,   // Lawson RK4 stages
    COL_FILTER = 5,   // Y -> multiplier * 1_S -> Y   (precondition)
    COL_FROM_STATE = 6,   // compact state -> derived fields (no input transform)
    COL_ADJ_C = 7, COL_ADJ_B = 8, COL_ADJ_A = 9, COL_ADJ_N = 10,  // adjoint stages
    COL_ADJ_SRC = 11, // terminal source -> lambda_H
    COL_FIRST_GUESS = 12, // probe velocities (u, v grids) -> band-limited vorticity
    COL_ADJ_NSRC = 13     // adjoint stage n at an observed step: two more inputs (residual sources)
};

struct ColArgs {
    const cd* yin[4];        // inputs (Y layout)
    int nin;                 // adjoint modes: number of inputs
    int inmul[4];            // adjoint modes: InMul per input
    cd* yout[4];             // derived outputs (Y layout)
    int nout;
    int fields[4];           // FieldKind per output
    cd* omega;               // compact state (rw)
    cd* acc;                 // compact RK4 accumulator (rw)
    cd* lam;                 // compact adjoint lambda_{n+1} / lambda_n
    cd* omb;                 // compact adjoint accumulator omega-bar
    cd* ckpt;                // optional compact checkpoint (write)
    const cd* state_in;      // COL_FROM_STATE input
    const double* invk2;     // [KY][KXP] 1/|k|^2 on S, 0 elsewhere
    const double* ex2;       // [KXP] exp(-(nu kx^2 + mu) h/2)
    const double* ey2;       // [KY]  exp(-nu ky^2 h/2)
    const double* mult;      // [B?][KY][KXP] real multiplier (COL_FILTER)
    const double* scale;     // [B] gradient scale (final adjoint output) or null
    const cd* tw;            // twiddles exp(-2 pi i m/N)
    double h;                // time step
    double forcing;          // value of the curl-force spectrum at (0, +-n_f)
    int nf;                  // n_f (0 = none or outside the band)
    int final_out;           // adjoint: emit the gradient field instead of Lambda
    int mult_per_member;     // COL_FILTER: multiplier table per member
    int lowpass;             // COL_FIRST_GUESS: keep |kx|, |ky| <= lowpass
    cd* omega_out;           // COL_D: the new state, in a buffer other than omega (null: in place)
    int split;               // set by the launcher: the derived fields of a column are shared out
                             // over this many workgroups (blockIdx.z, round robin); the first also
                             // writes the compact outputs
};

struct RowObs {
    int slot;                // observation slot, -1 = none
    int stride, M, n_times;
    const double* values;    // [B][n_times][2][M][M] or null
    double* obs_out;         // [B][n_times][2][M][M] or null
    double* jpart;           // [B][n_times][M] or null
    int imp_x, imp_y;        // impulse source (row_src mode 1)
};

struct RowArgs {
    const cd* yin[6];
    cd* yout[4];
    const double* phys_in;
    double* phys_out;
    const cd* tw;
    RowObs obs;
};

// Per-grid-size launchers, instantiated in kern_<N>.hip.
template <int N>
struct Launch {
    static hipError_t row_r2c(const Dims& d, const double* in, cd* out, const cd* tw, hipStream_t s);
    static hipError_t row_c2r(const Dims& d, const cd* in, double* out, const cd* tw, hipStream_t s);
    static hipError_t row_nl(const Dims& d, const RowArgs& a, hipStream_t s);
    static hipError_t row_obs(const Dims& d, const RowArgs& a, hipStream_t s);
    static hipError_t row_adj(const Dims& d, const RowArgs& a, hipStream_t s);
    static hipError_t row_src(const Dims& d, const RowArgs& a, int impulse, hipStream_t s);
    static hipError_t col(const Dims& d, int mode, const ColArgs& a, hipStream_t s);
    static int threads(int var);
};

// Threads per transform for grid size N and plan variant var.
int fft_threads(int N, int var);

// launchers (kernels.hip)
hipError_t launch_row_r2c(const Dims& d, const double* in, cd* out, const cd* tw, hipStream_t s);
hipError_t launch_row_c2r(const Dims& d, const cd* in, double* out, const cd* tw, hipStream_t s);
hipError_t launch_row_nl(const Dims& d, const RowArgs& a, hipStream_t s);
hipError_t launch_row_obs(const Dims& d, const RowArgs& a, hipStream_t s);
hipError_t launch_row_adj(const Dims& d, const RowArgs& a, hipStream_t s);
hipError_t launch_row_src(const Dims& d, const RowArgs& a, int impulse, hipStream_t s);
hipError_t launch_col(const Dims& d, int mode, const ColArgs& a, hipStream_t s);

// small kernels (misc.hip)
hipError_t launch_reduce_j(int B, int n_rows, const double* jpart, double* J, hipStream_t s);
hipError_t launch_fill(double* p, double v, size_t n, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t s);
hipError_t launch_make_mult(const Dims& d, int kind, int metric, double param, double power,
                            double* mult, hipStream_t s);
hipError_t launch_init_spectrum(const Dims& d, const uint64_t* seeds, int kind, double k0,
                                cd* state, hipStream_t s);
hipError_t launch_state_norm(const Dims& d, const cd* state, int kind, double* out, hipStream_t s);
hipError_t launch_state_scale(const Dims& d, cd* state, int kind, double target, const double* norm,
                              hipStream_t s);
hipError_t launch_shells(const Dims& d, const cd* lam, const int* shell_start, const int* shell_modes,
                         int n_shells, double* out, size_t out_stride, hipStream_t s);
// batched vector algebra over B members of length n (deterministic reductions)
hipError_t launch_dot(int B, size_t n, const double* x, const double* y, double* out, double* partial,
                      hipStream_t s);
hipError_t launch_axpy(int B, size_t n, const double* alpha, double alpha_scale, const double* x,
                       double* y, const int* active, hipStream_t s);
hipError_t launch_axpby(int B, size_t n, const double* alpha, double alpha_scale, const double* x,
                        const double* beta, double beta_scale, const double* y, double* z,
                        const int* active, hipStream_t s);
hipError_t launch_scal_copy(int B, size_t n, const double* alpha, const double* x, double* y,
                            hipStream_t s);
hipError_t launch_nonfinite(int B, size_t n, const double* x, int* flags, hipStream_t s);
hipError_t launch_scatter_probes(int B, int N, int stride, const double* probes, double* grid_u, double* grid_v,
                                 hipStream_t s);
// out[b] = scale * sum_k 1/2 |state_hat_b|^2 / N^4 over the band (= scale * grid mean of the field's
// square / 2 by Parseval)
hipError_t launch_state_energy(const Dims& d, const cd* state, double scale, double* out, hipStream_t s);
// ensemble statistics: add one batch at one row (adjoint step), and the final statistics
hipError_t launch_ens_accumulate(const Dims& d, const cd* lam, cd* lambda_sum_row, const double* shells_row,
                                 size_t shells_stride, int n_shells, double* shell_sum_row, double* etot_scratch,
                                 double* energy_sum_row, hipStream_t s);
hipError_t launch_ens_stats(const Dims& d, int rows, int n_shells, double inv_count, const cd* lambda_sum,
                            const double* shell_sum, const double* energy_sum, const int* shell_start,
                            const int* shell_modes, double* mean_energy, double* energy_of_mean, double* total_mean,
                            double* total_of_mean, double* snr, hipStream_t s);
hipError_t launch_shell_growth(int B, int rows, int n_shells, const double* shells, double dt, double tau_min,
                               double tau_max, double* mean_out, double* rate_out, hipStream_t s);

// batched L-BFGS scalars on the device (misc.hip): ring slot p of member b at [p * B + b]
hipError_t launch_fill_int(int* p, int v, size_t n, hipStream_t s);
hipError_t launch_lbfgs_first(int B, int sl, const double* dots, const int* ok, const double* rho, double* al,
                              double* coef, hipStream_t s);
hipError_t launch_lbfgs_gamma(int B, int m, int lo, int hi, const int* ok, const double* gam, double* coef,
                              hipStream_t s);
hipError_t launch_lbfgs_second(int B, int sl, const double* dots, const int* ok, const double* rho, const double* al,
                               double* coef, hipStream_t s);
hipError_t launch_lbfgs_direction(int B, int m, int lo, int hi, int use_pairs, double* gd, const double* gg,
                                  const double* J, int* ok, int* reset, double* alpha, const int* running, int* pend,
                                  int* acc, hipStream_t s);
hipError_t launch_lbfgs_armijo(int B, const double* Jtrial, const double* J0, double* alpha, const double* gd,
                               int* pend, int* acc, double* Jt, int* counts, hipStream_t s);
hipError_t launch_lbfgs_close(int B, const int* pend, const int* acc, const double* Jt, int* running, double* J,
                              hipStream_t s);
hipError_t launch_lbfgs_pair(int B, int sl, const double* sy, const double* ss, const double* yy, const int* acc,
                             int* ok, double* rho, double* gam, hipStream_t s);

constexpr int DOT_BLOCKS = 64;   // partial sums per member in launch_dot

// Events that the next row, column or pipelined-row kernel launched on this
// thread records as part of its own dispatch (start and end of that kernel,
// not of the packets around it).  Set by the launch timer; one launch
// consumes them and marks them used.
struct DispatchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
DispatchEvents& dispatch_events();

}  // namespace pa
