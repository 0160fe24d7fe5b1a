// misc.hip -- small kernels: deterministic reductions, batched vector algebra
// for the optimiser, preconditioner multipliers, seeded initial spectra and
// adjoint shell energies.  Every reduction runs in a fixed order (no atomics),
// so results are bitwise reproducible and independent of the batch size.
#include "kernels.hpp"

namespace pa {

__global__ void reduce_j_kernel(int B, int n_rows, const double* __restrict__ jpart, double* __restrict__ J) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    const double* p = jpart + (size_t)b * n_rows;
    for (int i = 0; i < n_rows; ++i) s += p[i];
    J[b] = s;
}
hipError_t launch_reduce_j(int B, int n_rows, const double* jpart, double* J, hipStream_t s) {
    hipLaunchKernelGGL(reduce_j_kernel, dim3((B + 63) / 64), dim3(64), 0, s, B, n_rows, jpart, J);
    return hipGetLastError();
}

__global__ void fill_kernel(double* __restrict__ p, double v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
hipError_t launch_fill(double* p, double v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t s) {
    if (n == 0 || dst == src) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

// (m^2 W)^power on the band, 0 elsewhere.  kind: 0 identity, 1 exp(-p|k|),
// 2 |k|^(-2p), 3 exp(-p|k|^2); metric 0 velocity (m^2 = |k|^2), 1 vorticity.
__global__ void make_mult_kernel(Dims d, int kind, int metric, double param, double power,
                                 double* __restrict__ mult) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.KY * d.KXP) return;
    const int r = i / d.KXP, kx = i % d.KXP;
    const int ky = (r <= d.K) ? r : r - d.KY;
    const double k2 = (double)kx * kx + (double)ky * ky;
    if (kx > d.K || k2 == 0.0) { mult[i] = 0.0; return; }
    const double kap = sqrt(k2);
    double W = 1.0;
    if (kind == 1) W = exp(-param * kap);
    else if (kind == 2) W = pow(kap, -2.0 * param);
    else if (kind == 3) W = exp(-param * k2);
    const double base = (metric == 0 ? k2 : metric == 2 ? k2 * k2 : 1.0) * W;
    mult[i] = pow(base, power);
}
hipError_t launch_make_mult(const Dims& d, int kind, int metric, double param, double power, double* mult,
                            hipStream_t s) {
    const int n = d.KY * d.KXP;
    hipLaunchKernelGGL(make_mult_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, kind, metric, param,
                       power, mult);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fields --
// SplitMix64 (Steele, Lea & Flood 2014): n-th output of the stream seeded
// with `seed` is mix64(seed + n * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double unit_draw(uint64_t seed, int kx, int ky, int stream) {
    const uint64_t n = 1ull + (uint64_t)stream + 4ull * ((uint64_t)(kx + 2048) + 4096ull * (uint64_t)(ky + 2048));
    return (double)(splitmix64(seed, n) >> 11) * 0x1.0p-53;
}

__global__ void init_spectrum_kernel(Dims d, const uint64_t* __restrict__ seeds, int kind, double k0,
                                     cd* __restrict__ state) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= d.KY * d.KXP) return;
    const int r = i / d.KXP, kx = i % d.KXP;
    const int ky = (r <= d.K) ? r : r - d.KY;
    cd out = czero();
    if (kx <= d.K && !(kx == 0 && ky == 0)) {
        const bool inside = (ky > 0) || (ky == 0 && kx > 0);
        const int rx = inside ? kx : -kx, ry = inside ? ky : -ky;
        const uint64_t seed = seeds[b];
        const double kap = sqrt((double)kx * kx + (double)ky * ky);
        const double twopi = 6.283185307179586476925286766559;
        double zr, zi, amp;
        if (kind == 0) {
            const double U = unit_draw(seed, rx, ry, 0);
            zr = cos(twopi * U);
            zi = sin(twopi * U);
        } else {
            const double U1 = unit_draw(seed, rx, ry, 1);
            const double U2 = unit_draw(seed, rx, ry, 2);
            const double rad = sqrt(-2.0 * log(1.0 - U1));
            zr = rad * cos(twopi * U2) / sqrt(2.0);
            zi = rad * sin(twopi * U2) / sqrt(2.0);
        }
        if (kind == 2) {
            amp = 1.0;
        } else {
            const double q = kap / k0;
            amp = sqrt(kap * (kap * kap * kap * kap * exp(-2.0 * q * q)));
        }
        out = mk(amp * zr, inside ? amp * zi : -amp * zi);
    }
    state[(size_t)b * d.KY * d.KXP + i] = out;
}
hipError_t launch_init_spectrum(const Dims& d, const uint64_t* seeds, int kind, double k0, cd* state,
                                hipStream_t s) {
    const int n = d.KY * d.KXP;
    hipLaunchKernelGGL(init_spectrum_kernel, dim3((n + 255) / 256, d.B), dim3(256), 0, s, d, seeds, kind, k0,
                       state);
    return hipGetLastError();
}

// kind 0/1: sum over the full spectrum of |w|^2 / |k|^2; kind 2: of |w|^2.
// One block per member, fixed-order tree.
__global__ void state_norm_kernel(Dims d, const cd* __restrict__ state, int kind, double* __restrict__ out) {
    __shared__ double sh[256];
    const int b = blockIdx.x;
    const cd* st = state + (size_t)b * d.KY * d.KXP;
    double acc = 0.0;
    for (int i = threadIdx.x; i < d.KY * d.KXP; i += blockDim.x) {
        const int r = i / d.KXP, kx = i % d.KXP;
        if (kx > d.K) continue;
        const int ky = (r <= d.K) ? r : r - d.KY;
        const double k2 = (double)kx * kx + (double)ky * ky;
        if (k2 == 0.0) continue;
        const double wgt = kx > 0 ? 2.0 : 1.0;
        const double a2 = st[i].x * st[i].x + st[i].y * st[i].y;
        acc += wgt * (kind == 2 ? a2 : a2 / k2);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = sh[0];
}
hipError_t launch_state_norm(const Dims& d, const cd* state, int kind, double* out, hipStream_t s) {
    hipLaunchKernelGGL(state_norm_kernel, dim3(d.B), dim3(256), 0, s, d, state, kind, out);
    return hipGetLastError();
}

__global__ void state_scale_kernel(Dims d, cd* __restrict__ state, int kind, double target,
                                   const double* __restrict__ norm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= d.KY * d.KXP) return;
    const double n4 = (double)d.N * d.N * (double)d.N * d.N;
    double f;
    if (kind == 2) f = target / (sqrt(norm[b]) / ((double)d.N * d.N));
    else f = sqrt(target / (0.5 * norm[b] / n4));
    cd& v = state[(size_t)b * d.KY * d.KXP + i];
    v = cscale(v, f);
}
hipError_t launch_state_scale(const Dims& d, cd* state, int kind, double target, const double* norm,
                              hipStream_t s) {
    const int n = d.KY * d.KXP;
    hipLaunchKernelGGL(state_scale_kernel, dim3((n + 255) / 256, d.B), dim3(256), 0, s, d, state, kind,
                       target, norm);
    return hipGetLastError();
}

// Shell energies 1/2 |k|^2 |lam|^2 / N^4 per unit-width shell k = 1..n_shells.
// shell_modes lists compact indices r*KXP + kx grouped by shell (CSR with
// shell_start).  One wavefront per (shell, member), so the whole grid is
// resident at once.  Each lane takes up to SHELL_BATCH modes of the shell per
// pass and issues all their index loads, then all their value loads, before
// adding: a pass costs two memory latencies (one pass covers any shell of
// 256^2).  Lanes add in a fixed stride and a fixed butterfly.
// A shell is an annulus that meets most rows in one or two modes, so its
// gather uses a small part of each cache line; the other shells of the member
// use the rest.  Workgroups are dealt to the XCDs in turn, so workgroup w is
// mapped to member (w mod XCDS) + XCDS * (w / (XCDS n_shells)): all shells of
// a member run on one XCD and share its L2, which holds the few members of
// that XCD.
constexpr int SHELL_THREADS = 64;
constexpr int SHELL_BATCH = 8;
constexpr int SHELL_XCDS = 8;   // accelerator complex dies of the device
__global__ void __launch_bounds__(SHELL_THREADS) shells_kernel(Dims d, const cd* __restrict__ lam,
                                                               const int* __restrict__ start,
                                                               const int* __restrict__ modes, int n_shells,
                                                               double* __restrict__ out, size_t out_stride) {
    const int w = blockIdx.x;
    const int q = w / SHELL_XCDS;
    const int b = w % SHELL_XCDS + SHELL_XCDS * (q / n_shells);
    const int k = q % n_shells;
    if (b >= d.B) return;   // the last group of members may be partial
    const int lane = threadIdx.x;
    const cd* __restrict__ l = lam + (size_t)b * d.KY * d.KXP;
    const int lo = start[k], hi = start[k + 1];
    double s = 0.0;
    for (int base = lo; base < hi; base += SHELL_BATCH * SHELL_THREADS) {
        int mb[SHELL_BATCH];
        cd vb[SHELL_BATCH];
#pragma unroll
        for (int u = 0; u < SHELL_BATCH; ++u) {
            const int i = base + u * SHELL_THREADS + lane;
            mb[u] = i < hi ? modes[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < SHELL_BATCH; ++u) vb[u] = mb[u] >= 0 ? l[mb[u]] : cd{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < SHELL_BATCH; ++u) {
            if (mb[u] < 0) continue;
            const int r = mb[u] / d.KXP, kx = mb[u] - r * d.KXP;
            const int ky = (r <= d.K) ? r : r - d.KY;
            const double k2 = (double)kx * kx + (double)ky * ky;
            const double wgt = kx > 0 ? 2.0 : 1.0;
            s += wgt * 0.5 * k2 * (vb[u].x * vb[u].x + vb[u].y * vb[u].y);
        }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const double n4 = (double)d.N * d.N * (double)d.N * d.N;
        out[(size_t)b * out_stride + k] = s / n4;
    }
}
hipError_t launch_shells(const Dims& d, const cd* lam, const int* shell_start, const int* shell_modes,
                         int n_shells, double* out, size_t out_stride, hipStream_t s) {
    if (!lam || !shell_start || !shell_modes || !out || n_shells < 1) return hipErrorInvalidValue;
    const size_t groups = (size_t)SHELL_XCDS * n_shells * ((d.B + SHELL_XCDS - 1) / SHELL_XCDS);
    if (groups > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(shells_kernel, dim3((unsigned)groups), dim3(SHELL_THREADS), 0, s, d, lam, shell_start,
                       shell_modes, n_shells, out, out_stride);
    return hipGetLastError();
}

// ------------------------------------------------- ensemble statistics --
// Accumulators over an ensemble split into batches: members are added one at
// a time in member order onto the running sum, so any split into batches
// gives bitwise the same sums.  Padding columns kx > Kc are never touched.

__global__ void ens_lambda_sum_kernel(Dims d, const cd* __restrict__ lam, cd* __restrict__ sum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // compact index r * KXP + kx
    if (i >= d.KY * d.KXP || i % d.KXP > d.K) return;
    const size_t SC = (size_t)d.KY * d.KXP;
    cd acc = sum[i];
    for (int b = 0; b < d.B; ++b) {
        const cd v = lam[(size_t)b * SC + i];
        acc.x += v.x;
        acc.y += v.y;
    }
    sum[i] = acc;
}

// acc[k] += v[0 * stride + k] + v[1 * stride + k] + ... (member order), k < n
__global__ void ens_scalar_sum_kernel(int B, const double* __restrict__ v, size_t stride, int n,
                                      double* __restrict__ acc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double a = acc[k];
    for (int b = 0; b < B; ++b) a += v[(size_t)b * stride + k];
    acc[k] = a;
}

// sum_k 1/2 |k|^(2 p) |lam_hat|^2 / N^4 over the band of each of d.B compact
// states (kx > 0 counted twice for the Hermitian half), times scale, for p =
// k2pow in {0, 1}: with p = 1 the adjoint velocity energy, with p = 0 half
// the grid mean of the field's square.  One workgroup per state,
// fixed-order tree.
constexpr int ETOT_THREADS = 256;
__global__ void __launch_bounds__(ETOT_THREADS) energy_total_kernel(Dims d, const cd* __restrict__ lam, double scale,
                                                                    double* __restrict__ out, int k2pow) {
    __shared__ double sh[ETOT_THREADS];
    const int b = blockIdx.x;
    const size_t SC = (size_t)d.KY * d.KXP;
    const cd* l = lam + (size_t)b * SC;
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)SC; i += ETOT_THREADS) {
        const int r = i / d.KXP, kx = i % d.KXP;
        if (kx > d.K) continue;
        const int ky = (r <= d.K) ? r : r - d.KY;
        const double k2 = (double)kx * kx + (double)ky * ky;
        const double wgt = kx > 0 ? 2.0 : 1.0;
        s += wgt * 0.5 * (k2pow ? k2 : 1.0) * (l[i].x * l[i].x + l[i].y * l[i].y);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = ETOT_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n4 = (double)d.N * d.N * (double)d.N * d.N;
        out[b] = scale * sh[0] / n4;
    }
}

// Per row: mean shell energy, energy of the mean (from the shells of the
// member sum), their totals and the ratio of the totals.
__global__ void ens_finish_kernel(int rows, int n_shells, double inv_count, const double* __restrict__ shell_sum,
                                  const double* __restrict__ energy_sum, double* __restrict__ mean_energy,
                                  double* __restrict__ energy_of_mean, double* __restrict__ total_mean,
                                  double* __restrict__ total_of_mean, double* __restrict__ snr) {
    const int row = blockIdx.x;
    const double c2 = inv_count * inv_count;
    for (int k = threadIdx.x; k < n_shells; k += blockDim.x) {
        const size_t i = (size_t)row * n_shells + k;
        mean_energy[i] = shell_sum[i] * inv_count;
        energy_of_mean[i] *= c2;
    }
    if (threadIdx.x == 0) {
        const double tm = energy_sum[row] * inv_count;
        const double te = total_of_mean[row] * c2;
        total_mean[row] = tm;
        total_of_mean[row] = te;
        snr[row] = tm > 0.0 ? te / tm : NAN;
    }
}

hipError_t launch_state_energy(const Dims& d, const cd* state, double scale, double* out, hipStream_t s) {
    if (!state || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(energy_total_kernel, dim3(d.B), dim3(ETOT_THREADS), 0, s, d, state, scale, out, 0);
    return hipGetLastError();
}

hipError_t launch_ens_accumulate(const Dims& d, const cd* lam, cd* lambda_sum_row, const double* shells_row,
                                 size_t shells_stride, int n_shells, double* shell_sum_row, double* etot_scratch,
                                 double* energy_sum_row, hipStream_t s) {
    if (!lam || !lambda_sum_row || !shells_row || !shell_sum_row || !etot_scratch || !energy_sum_row)
        return hipErrorInvalidValue;
    const int n = d.KY * d.KXP;
    hipLaunchKernelGGL(ens_lambda_sum_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, lam, lambda_sum_row);
    hipLaunchKernelGGL(ens_scalar_sum_kernel, dim3((n_shells + 63) / 64), dim3(64), 0, s, d.B, shells_row,
                       shells_stride, n_shells, shell_sum_row);
    hipLaunchKernelGGL(energy_total_kernel, dim3(d.B), dim3(ETOT_THREADS), 0, s, d, lam, 1.0, etot_scratch, 1);
    hipLaunchKernelGGL(ens_scalar_sum_kernel, dim3(1), dim3(64), 0, s, d.B, etot_scratch, (size_t)1, 1,
                       energy_sum_row);
    return hipGetLastError();
}

hipError_t launch_ens_stats(const Dims& d, int rows, int n_shells, double inv_count, const cd* lambda_sum,
                            const double* shell_sum, const double* energy_sum, const int* shell_start,
                            const int* shell_modes, double* mean_energy, double* energy_of_mean, double* total_mean,
                            double* total_of_mean, double* snr, hipStream_t s) {
    if (!lambda_sum || !shell_sum || !energy_sum || !mean_energy || !energy_of_mean || !total_mean ||
        !total_of_mean || !snr || rows < 1 || n_shells < 1)
        return hipErrorInvalidValue;
    Dims dr = d;
    dr.B = rows;   // the rows of the member sum take the place of members
    hipError_t e = launch_shells(dr, lambda_sum, shell_start, shell_modes, n_shells, energy_of_mean,
                                 (size_t)n_shells, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(energy_total_kernel, dim3(rows), dim3(ETOT_THREADS), 0, s, dr, lambda_sum, 1.0, total_of_mean,
                       1);
    hipLaunchKernelGGL(ens_finish_kernel, dim3(rows), dim3(64), 0, s, rows, n_shells, inv_count, shell_sum,
                       energy_sum, mean_energy, energy_of_mean, total_mean, total_of_mean, snr);
    return hipGetLastError();
}

// ------------------------------------------------------- vector algebra --

__global__ void dot_partial_kernel(size_t n, const double* __restrict__ x, const double* __restrict__ y,
                                   double* __restrict__ partial) {
    __shared__ double sh[256];
    const int b = blockIdx.y;
    const size_t chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
    const size_t lo = blockIdx.x * chunk;
    const size_t hi = (lo + chunk < n) ? lo + chunk : n;
    const double* xb = x + (size_t)b * n;
    const double* yb = y + (size_t)b * n;
    double acc = 0.0;
    for (size_t i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += xb[i] * yb[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)b * DOT_BLOCKS + blockIdx.x] = sh[0];
}
__global__ void dot_final_kernel(int B, const double* __restrict__ partial, double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int i = 0; i < DOT_BLOCKS; ++i) s += partial[(size_t)b * DOT_BLOCKS + i];
    out[b] = s;
}
hipError_t launch_dot(int B, size_t n, const double* x, const double* y, double* out, double* partial,
                      hipStream_t s) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS, B), dim3(256), 0, s, n, x, y, partial);
    hipLaunchKernelGGL(dot_final_kernel, dim3((B + 63) / 64), dim3(64), 0, s, B, partial, out);
    return hipGetLastError();
}

// y[b] += alpha[b] * alpha_scale * x[b]  (members with active[b] == 0 untouched)
__global__ void axpy_kernel(size_t n, const double* __restrict__ alpha, double alpha_scale,
                            const double* __restrict__ x, double* __restrict__ y, const int* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double a = (alpha ? alpha[b] : 1.0) * alpha_scale;
    const double* xb = x + (size_t)b * n;
    double* yb = y + (size_t)b * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        yb[i] += a * xb[i];
}
hipError_t launch_axpy(int B, size_t n, const double* alpha, double alpha_scale, const double* x, double* y,
                       const int* active, hipStream_t s) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)blocks, B), dim3(256), 0, s, n, alpha, alpha_scale, x, y,
                       active);
    return hipGetLastError();
}

// z[b] = alpha[b]*as * x[b] + beta[b]*bs * y[b]   (null alpha/beta read as 1)
__global__ void axpby_kernel(size_t n, const double* __restrict__ alpha, double as, const double* __restrict__ x,
                             const double* __restrict__ beta, double bs, const double* __restrict__ y,
                             double* __restrict__ z, const int* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double a = (alpha ? alpha[b] : 1.0) * as;
    const double c = (beta ? beta[b] : 1.0) * bs;
    const double* xb = x + (size_t)b * n;
    const double* yb = y + (size_t)b * n;
    double* zb = z + (size_t)b * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        zb[i] = a * xb[i] + c * yb[i];
}
hipError_t launch_axpby(int B, size_t n, const double* alpha, double alpha_scale, const double* x,
                        const double* beta, double beta_scale, const double* y, double* z, const int* active,
                        hipStream_t s) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)blocks, B), dim3(256), 0, s, n, alpha, alpha_scale, x, beta,
                       beta_scale, y, z, active);
    return hipGetLastError();
}

// y[b] = alpha[b] * x[b]
__global__ void scal_copy_kernel(size_t n, const double* __restrict__ alpha, const double* __restrict__ x,
                                 double* __restrict__ y) {
    const int b = blockIdx.y;
    const double a = alpha[b];
    const double* xb = x + (size_t)b * n;
    double* yb = y + (size_t)b * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        yb[i] = a * xb[i];
}
hipError_t launch_scal_copy(int B, size_t n, const double* alpha, const double* x, double* y, hipStream_t s) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(scal_copy_kernel, dim3((unsigned)blocks, B), dim3(256), 0, s, n, alpha, x, y);
    return hipGetLastError();
}

// flags[b] = 1 if any entry of member b is not finite (flags must start at 0).
__global__ void nonfinite_kernel(size_t n, const double* __restrict__ x, int* __restrict__ flags) {
    const int b = blockIdx.y;
    const double* xb = x + (size_t)b * n;
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(xb[i])) bad = 1;
    if (bad) flags[b] = 1;
}
hipError_t launch_nonfinite(int B, size_t n, const double* x, int* flags, hipStream_t s) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks, B), dim3(256), 0, s, n, x, flags);
    return hipGetLastError();
}

// Probe velocities [B][2][M][M] scattered onto zero grids [B][N][N] at (i s, j s),
// times s^2: the unnormalised transform of that grid restricted to |k| < M/2
// is (N/M)^2 times the coarse transform of the probes.
__global__ void scatter_probes_kernel(int N, int stride, const double* __restrict__ probes, double* __restrict__ gu,
                                      double* __restrict__ gv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= N * N) return;
    const int y = i / N, x = i % N;
    const int M = N / stride;
    double u = 0.0, v = 0.0;
    if (y % stride == 0 && x % stride == 0) {
        const size_t base = (size_t)b * 2 * M * M + (size_t)(y / stride) * M + (x / stride);
        const double s2 = (double)stride * stride;
        u = s2 * probes[base];
        v = s2 * probes[base + (size_t)M * M];
    }
    gu[(size_t)b * N * N + i] = u;
    gv[(size_t)b * N * N + i] = v;
}
hipError_t launch_scatter_probes(int B, int N, int stride, const double* probes, double* grid_u, double* grid_v,
                                 hipStream_t s) {
    if (!probes || !grid_u || !grid_v || stride < 1 || N % stride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scatter_probes_kernel, dim3((N * N + 255) / 256, B), dim3(256), 0, s, N, stride, probes,
                       grid_u, grid_v);
    return hipGetLastError();
}

// Ensemble mean of shell energies and least-squares growth rate per shell:
// mean[n][k] = (1/B) sum_b shells[b][n][k];  rate[k] = slope of ln mean[n][k]
// against tau = n dt over tau in [tau_min, tau_max] (NaN when a value is not
// positive or fewer than two rows fall in the window).  One thread per shell.
__global__ void shell_growth_kernel(int B, int rows, int n_shells, const double* __restrict__ shells, double dt,
                                    double tau_min, double tau_max, double* __restrict__ mean,
                                    double* __restrict__ rate) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_shells) return;
    double st = 0.0, sy = 0.0, stt = 0.0, sty = 0.0;
    int cnt = 0;
    bool ok = true;
    for (int n = 0; n < rows; ++n) {
        double m = 0.0;
        for (int b = 0; b < B; ++b) m += shells[((size_t)b * rows + n) * n_shells + k];
        m /= (double)B;
        if (mean) mean[(size_t)n * n_shells + k] = m;
        const double tau = n * dt;
        if (tau >= tau_min - 1e-12 && tau <= tau_max + 1e-12) {
            if (!(m > 0.0)) { ok = false; continue; }
            const double ly = log(m);
            st += tau; sy += ly; stt += tau * tau; sty += tau * ly;
            ++cnt;
        }
    }
    double r = NAN;
    if (ok && cnt >= 2) {
        const double tm = st / cnt, ym = sy / cnt;
        r = (sty - cnt * tm * ym) / (stt - cnt * tm * tm);
    }
    rate[k] = r;
}
hipError_t launch_shell_growth(int B, int rows, int n_shells, const double* shells, double dt, double tau_min,
                               double tau_max, double* mean_out, double* rate_out, hipStream_t s) {
    if (!shells || !rate_out || B < 1 || rows < 1 || n_shells < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(shell_growth_kernel, dim3((n_shells + 63) / 64), dim3(64), 0, s, B, rows, n_shells, shells, dt,
                       tau_min, tau_max, mean_out, rate_out);
    return hipGetLastError();
}

// ------------------------------------------------- L-BFGS on the device --
// The per-member scalars of the batched L-BFGS / steepest-descent loop live
// in device arrays; these kernels take the decisions the recursion needs
// (two-loop coefficients, memory reset, trial step, Armijo test, curvature
// test) elementwise over the members, in the same operations and order as a
// host loop would (no contraction into fused multiply-adds), so the iterates
// do not depend on where the scalars live.  Ring slot p of member b is
// [p * B + b]; pairs p in [lo, hi) of the ring are the stored window.

namespace {
__device__ __forceinline__ bool window_has_pair(const int* ok, int B, int b, int m, int lo, int hi) {
    for (int p = lo; p < hi; ++p)
        if (ok[(size_t)(p % m) * B + b]) return true;
    return false;
}
}  // namespace

__global__ void fill_int_kernel(int* __restrict__ p, int v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
hipError_t launch_fill_int(int* p, int v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// first loop, pair slot sl: al = rho (s . q) where the member holds the pair, else 0; coef = -al
__global__ void lbfgs_first_kernel(int B, int sl, const double* __restrict__ dots, const int* __restrict__ ok,
                                   const double* __restrict__ rho, double* __restrict__ al, double* __restrict__ coef) {
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const size_t i = (size_t)sl * B + b;
    const double a = ok[i] ? rho[i] * dots[b] : 0.0;
    al[i] = a;
    coef[b] = -a;
}
// H0 = gamma I from each member's newest stored pair of the window, else 1
__global__ void lbfgs_gamma_kernel(int B, int m, int lo, int hi, const int* __restrict__ ok,
                                   const double* __restrict__ gam, double* __restrict__ coef) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double g = 1.0;
    for (int p = hi - 1; p >= lo; --p) {
        const size_t i = (size_t)(p % m) * B + b;
        if (ok[i]) {
            g = gam[i];
            break;
        }
    }
    coef[b] = g;
}
// second loop, pair slot sl: coef = al - rho (y . r) where the member holds the pair, else 0
__global__ void lbfgs_second_kernel(int B, int sl, const double* __restrict__ dots, const int* __restrict__ ok,
                                    const double* __restrict__ rho, const double* __restrict__ al,
                                    double* __restrict__ coef) {
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const size_t i = (size_t)sl * B + b;
    coef[b] = ok[i] ? al[i] - rho[i] * dots[b] : 0.0;
}
// Search-direction checks from gd = g . d and gg = g . g: a member with stored
// pairs whose d is not a descent direction drops its pairs (reset = 1, d is
// then set to -g) and takes gd = -gg; the trial step is 1 with pairs, else
// J / gg.  Opens the line search: pending = running, accepted = 0.
__global__ void lbfgs_direction_kernel(int B, int m, int lo, int hi, int use_pairs, double* __restrict__ gd,
                                       const double* __restrict__ gg, const double* __restrict__ J,
                                       int* __restrict__ ok, int* __restrict__ reset, double* __restrict__ alpha,
                                       const int* __restrict__ running, int* __restrict__ pend,
                                       int* __restrict__ acc) {
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    bool mem = use_pairs && window_has_pair(ok, B, b, m, lo, hi);
    int r = 0;
    if (mem && gd[b] >= 0.0) {
        r = 1;
        for (int s = 0; s < m; ++s) ok[(size_t)s * B + b] = 0;
        mem = false;
        gd[b] = -gg[b];
    }
    reset[b] = r;
    alpha[b] = mem ? 1.0 : J[b] / gg[b];
    pend[b] = running[b];
    acc[b] = 0;
}
// Armijo test of one trial for the pending members: accept (cost kept in Jt)
// if J <= J0 + c1 alpha gd, else halve alpha.  One block counts the members
// still pending and those accepted into counts[0..1].
__global__ void lbfgs_armijo_kernel(int B, const double* __restrict__ Jtrial, const double* __restrict__ J0,
                                    double* __restrict__ alpha, const double* __restrict__ gd, int* __restrict__ pend,
                                    int* __restrict__ acc, double* __restrict__ Jt, int* __restrict__ counts) {
#pragma clang fp contract(off)
    __shared__ int np[256], na[256];
    int cp = 0, ca = 0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        if (pend[b]) {
            if (Jtrial[b] <= J0[b] + 1e-4 * alpha[b] * gd[b]) {
                pend[b] = 0;
                acc[b] = 1;
                Jt[b] = Jtrial[b];
            } else {
                alpha[b] *= 0.5;
            }
        }
        cp += pend[b];
        ca += acc[b];
    }
    np[threadIdx.x] = cp;
    na[threadIdx.x] = ca;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            np[threadIdx.x] += np[threadIdx.x + w];
            na[threadIdx.x] += na[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[0] = np[0];
        counts[1] = na[0];
    }
}
// After the line search: members still pending failed (running = 0); the
// accepted ones take their trial cost.
__global__ void lbfgs_close_kernel(int B, const int* __restrict__ pend, const int* __restrict__ acc,
                                   const double* __restrict__ Jt, int* __restrict__ running, double* __restrict__ J) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (pend[b]) running[b] = 0;
    if (acc[b]) J[b] = Jt[b];
}
// Curvature test of the new pair in slot sl (sy, ss, yy = s.y, s.s, y.y): kept
// if the member accepted its step and sy > 1e-10 |s| |y|.
__global__ void lbfgs_pair_kernel(int B, int sl, const double* __restrict__ sy, const double* __restrict__ ss,
                                  const double* __restrict__ yy, const int* __restrict__ acc, int* __restrict__ ok,
                                  double* __restrict__ rho, double* __restrict__ gam) {
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const size_t i = (size_t)sl * B + b;
    const int k = acc[b] && sy[b] > 1e-10 * sqrt(ss[b]) * sqrt(yy[b]);
    ok[i] = k;
    rho[i] = k ? 1.0 / sy[b] : 0.0;
    gam[i] = k ? sy[b] / yy[b] : 1.0;
}

static dim3 member_grid(int B) { return dim3((unsigned)((B + 255) / 256)); }

hipError_t launch_lbfgs_first(int B, int sl, const double* dots, const int* ok, const double* rho, double* al,
                              double* coef, hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_first_kernel, member_grid(B), dim3(256), 0, s, B, sl, dots, ok, rho, al, coef);
    return hipGetLastError();
}
hipError_t launch_lbfgs_gamma(int B, int m, int lo, int hi, const int* ok, const double* gam, double* coef,
                              hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_gamma_kernel, member_grid(B), dim3(256), 0, s, B, m, lo, hi, ok, gam, coef);
    return hipGetLastError();
}
hipError_t launch_lbfgs_second(int B, int sl, const double* dots, const int* ok, const double* rho, const double* al,
                               double* coef, hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_second_kernel, member_grid(B), dim3(256), 0, s, B, sl, dots, ok, rho, al, coef);
    return hipGetLastError();
}
hipError_t launch_lbfgs_direction(int B, int m, int lo, int hi, int use_pairs, double* gd, const double* gg,
                                  const double* J, int* ok, int* reset, double* alpha, const int* running, int* pend,
                                  int* acc, hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_direction_kernel, member_grid(B), dim3(256), 0, s, B, m, lo, hi, use_pairs, gd, gg, J, ok,
                       reset, alpha, running, pend, acc);
    return hipGetLastError();
}
hipError_t launch_lbfgs_armijo(int B, const double* Jtrial, const double* J0, double* alpha, const double* gd,
                               int* pend, int* acc, double* Jt, int* counts, hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_armijo_kernel, dim3(1), dim3(256), 0, s, B, Jtrial, J0, alpha, gd, pend, acc, Jt, counts);
    return hipGetLastError();
}
hipError_t launch_lbfgs_close(int B, const int* pend, const int* acc, const double* Jt, int* running, double* J,
                              hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_close_kernel, member_grid(B), dim3(256), 0, s, B, pend, acc, Jt, running, J);
    return hipGetLastError();
}
hipError_t launch_lbfgs_pair(int B, int sl, const double* sy, const double* ss, const double* yy, const int* acc,
                             int* ok, double* rho, double* gam, hipStream_t s) {
    hipLaunchKernelGGL(lbfgs_pair_kernel, member_grid(B), dim3(256), 0, s, B, sl, sy, ss, yy, acc, ok, rho, gam);
    return hipGetLastError();
}

}  // namespace pa
