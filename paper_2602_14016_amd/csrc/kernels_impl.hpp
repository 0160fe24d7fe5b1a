// kernels_impl.hpp -- row (physical-space) and column (spectral-space) passes.
//
// Row pass: a team of T threads owns one grid row (or a pair of rows) of one
// member.  It rebuilds full complex rows from the stored half spectra
// (Hermitian extension, two real fields packed as re + i im), inverse
// transforms along x, forms the pointwise products of the method in
// registers, and forward transforms the products back, keeping kx <= Kc.
// Column pass: a team owns one kx column of one member; a workgroup holds CB
// adjacent columns so that every global access is a run of CB contiguous
// complex values.  It transforms along y, applies the spectral operators of
// the step mode by mode, and transforms the derived fields back along y.
//
// Included once per grid size by kern_<N>.hip, which instantiates Launch<N>.
#pragma once
#include <algorithm>
#include <atomic>

#include <hip/hip_ext.h>

#include "kernels.hpp"

namespace pa {

// Launch of a row or column kernel: with timing events pending on this
// thread, the dispatch itself records them (hipExtLaunchKernel), so the
// measured time is the kernel's and not that of separate event packets.
template <class F, class... Args>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
    DispatchEvents& e = dispatch_events();
    if (e.start && !e.used) {
        e.used = true;
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, s, e.start, e.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    }
}

// Global accesses as uniform base + 32-bit byte offset (element index << 4),
// so the backend can address with a scalar base and one 32-bit lane offset.
__device__ __forceinline__ cd ldc(const cd* base, unsigned i) {
    return *reinterpret_cast<const cd*>(reinterpret_cast<const char*>(base) + (i << 4));
}
__device__ __forceinline__ void stc(cd* base, unsigned i, cd v) {
    *reinterpret_cast<cd*>(reinterpret_cast<char*>(base) + (i << 4)) = v;
}

// The twiddle table is copied into LDS at kernel start, in the stage order of
// the plan: reads after a barrier are not hoisted out of loops, so they do
// not pin registers across the successive transforms of a kernel.
template <int N, int V>
__device__ __forceinline__ const cd* stage_twiddles(cd* lds_tw, const cd* __restrict__ tw) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) lds_tw[i] = tw[twiddle_source<N, V>(i)];
    lds_sync();
    return lds_tw;
}

// Row transforms of a kernel whose rows run several transforms with one set of
// twiddle factors per thread.  Plan (256, 2) (one row per wavefront, four
// values per lane) uses the wavefront-resident transform with lane swaps
// (fft256_wave), whose nine factors per thread come straight from the natural
// table; every other plan runs its Stockham stages with the factors of the
// stage-ordered table (staged in LDS by the workgroup) held in registers.
template <int N, int V>
__host__ __device__ constexpr bool wave256() { return N == 256 && V == 2; }

template <int N, int V>
struct RowTw {
    TwReg<N, V> r;
};
template <>
struct RowTw<256, 2> {
    Tw256 r;
};

template <int N, int V>
__device__ __forceinline__ void row_twiddles(RowTw<N, V>& tr, int t, const cd* __restrict__ tw_g, cd* tw_lds) {
    if constexpr (wave256<N, V>()) load_tw256(tr.r, t, tw_g);
    else load_twiddles<N, V>(tr.r, t, stage_twiddles<N, V>(tw_lds, tw_g));
}

template <int N, int V, bool INV, bool WL>
__device__ __forceinline__ void row_fft(cd* v, int t, cd* lds, const RowTw<N, V>& tr) {
    if constexpr (wave256<N, V>()) fft256_wave<INV>(v, t, lds, tr.r);
    else fft<N, V, INV, WL>(v, t, lds, tr.r);
}

// Retained band of a grid of size N: the 2/3 rule keeps |kx|, |ky| <= (N-1)/3.
template <int N>
__host__ __device__ constexpr int band() { return (N - 1) / 3; }
// Row pitch of the half-spectrum layouts: kx = 0..K padded to a multiple of 8.
template <int N>
__host__ __device__ constexpr int kx_pad() { return (band<N>() + 1 + 7) / 8 * 8; }

// Whether register slot m of a T-thread team (elements t + T m, t < T) can
// touch the band kx <= K or kx >= N - K; folded at compile time after
// unrolling, so slots that only see the de-aliased gap issue no loads.
template <int N, int V>
__device__ constexpr bool slot_in_band(int m) {
    constexpr int T = Plan<N, V>::T, K = band<N>();
    return T * m <= K || T * m + T - 1 >= N - K;
}
template <int N, int V>
__device__ constexpr bool slot_low(int m) { return Plan<N, V>::T * m <= band<N>(); }

// z = A_full[e] + i B_full[e] for the Hermitian extensions of half-spectrum
// rows A, B (only kx = 0..K stored, zero beyond): two rows of one field packed
// into one transform (the row pass from a single field to physical space).
// The kx = 0 entry of a real field's half spectrum is real; its imaginary
// round-off is discarded.  Branch-free: the load index is clamped to 0 off the
// band and the result selected, so the loads of all slots issue back to back
// instead of each waiting inside a divergent branch.
template <int N>
__device__ __forceinline__ cd herm_pair(const cd* __restrict__ A, const cd* __restrict__ B, int e) {
    constexpr int K = band<N>();
    const bool lo = e <= K, hi = e >= N - K;
    const unsigned k = lo ? (unsigned)e : (hi ? (unsigned)(N - e) : 0u);
    cd a = ldc(A, k), bb = ldc(B, k);
    if (e == 0) { a.y = 0.0; bb.y = 0.0; }
    if (hi) { a.y = -a.y; bb.y = -bb.y; }
    const cd z = mk(a.x - bb.y, a.y + bb.x);
    return (lo || hi) ? z : czero();
}

// Fills the E register slots of a team with the extension of (A, B).
template <int N, int V>
__device__ __forceinline__ void herm_load(cd* z, const cd* __restrict__ A, const cd* __restrict__ B, int t) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E;
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = slot_in_band<N, V>(m) ? herm_pair<N>(A, B, t + T * m) : czero();
}

// z = A_full[e] + i B_full[e] from the packed half spectra P = A + i B and
// Q = A - i B of one row: P[e] on the low band, conj(Q[N - e]) on the high
// band (the Hermitian extension of A and B), zero in the de-aliased gap.  Each
// register slot issues one load; which band its lanes can meet is known at
// compile time from the plan, so all-low and all-high slots carry no select.
template <int N, int V>
__device__ __forceinline__ void packed_load(cd* z, const cd* __restrict__ P, const cd* __restrict__ Q, int t) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E, K = band<N>();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + T * m;
        const bool all_lo = T * m + T - 1 <= K, all_hi = T * m >= N - K;
        const bool may_lo = T * m <= K, may_hi = T * m + T - 1 >= N - K;
        if (all_lo) {
            z[m] = ldc(P, (unsigned)e);
        } else if (all_hi) {
            const cd q = ldc(Q, (unsigned)(N - e));
            z[m] = mk(q.x, -q.y);
        } else if (may_lo && may_hi) {
            const bool lo = e <= K, hi = e >= N - K;
            const cd p = ldc(P, lo ? (unsigned)e : 0u), q = ldc(Q, hi ? (unsigned)(N - e) : 0u);
            z[m] = lo ? p : (hi ? mk(q.x, -q.y) : czero());
        } else if (may_lo) {
            const bool lo = e <= K;
            const cd p = ldc(P, lo ? (unsigned)e : 0u);
            z[m] = lo ? p : czero();
        } else if (may_hi) {
            const bool hi = e >= N - K;
            const cd q = ldc(Q, hi ? (unsigned)(N - e) : 0u);
            z[m] = hi ? mk(q.x, -q.y) : czero();
        } else {
            z[m] = czero();
        }
    }
}

// Forward transform z of a + i b (a, b real) is split into the half spectra
// of a and b:  Ahat[k] = (Z[k] + conj Z[N-k]) / 2,  Bhat[k] = (Z[k] - conj Z[N-k]) / (2i).
// Stores kx = 0..K of both.  Called by every thread of the workgroup.
template <int N, int V, bool WL>
__device__ __forceinline__ void split_store(const cd* z, int t, cd* lds, cd* __restrict__ outA,
                                            cd* __restrict__ outB) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E, K = band<N>();
#pragma unroll
    for (int m = 0; m < E; ++m) lds[lpos<N, V>(t + T * m)] = z[m];
    team_sync<WL>();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + T * m;
        if (slot_low<N, V>(m) && k <= K) {
            const cd zk = z[m];
            const cd zn = lds[lpos<N, V>((N - k) & (N - 1))];
            outA[k] = mk(0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y));
            outB[k] = mk(0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x));
        }
    }
    team_sync<WL>();
}

// Forward transform z of a + i b (a, b real) stored unsplit for k = 0..K:
// P[k] = Z[k] and Q[k] = conj(Z[N - k]), so that a_hat = (P + Q) / 2 and
// b_hat = (P - Q) / (2i) (the column pass forms them).  Each lane stores the
// values it holds: no exchange.
template <int N, int V>
__device__ __forceinline__ void pair_store(const cd* z, int t, cd* __restrict__ outP, cd* __restrict__ outQ) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E, K = band<N>();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + T * m;
        if (slot_low<N, V>(m) && k <= K) stc(outP, (unsigned)k, z[m]);
        const bool q_slot = m == 0 || T * m + T - 1 >= N - K;   // holds k = 0 or some k >= N - K
        const int kn = (N - k) & (N - 1);
        if (q_slot && kn <= K) stc(outQ, (unsigned)kn, mk(z[m].x, -z[m].y));
    }
}

// Team sum (fixed order) of one double per thread; result valid in thread t == 0.
template <int N, int V, bool WL>
__device__ __forceinline__ double team_sum(double v, int t, cd* lds) {
    constexpr int T = Plan<N, V>::T;
    lds[t] = mk(v, 0.0);
    team_sync<WL>();
    double s = 0.0;
    if (t == 0)
        for (int i = 0; i < T; ++i) s += lds[i].x;
    team_sync<WL>();
    return s;
}

// Observation of one velocity component c (0 = u, 1 = v) at (x, y): writes the
// model observation and returns the squared residual (0 off the probes).
__device__ __forceinline__ double observe_comp(const RowObs& o, int b, int y, int x, int comp, double val) {
    if ((y % o.stride) != 0 || (x % o.stride) != 0) return 0.0;
    const int i = x / o.stride, j = y / o.stride, M = o.M;
    const size_t idx = ((((size_t)b * o.n_times + o.slot) * 2) + comp) * M * M + (size_t)j * M + i;
    if (o.obs_out) o.obs_out[idx] = val;
    if (!o.values) return 0.0;
    const double r = val - o.values[idx];
    return r * r;
}

__device__ __forceinline__ void store_jpart(const RowObs& o, int b, int y, double s) {
    if (o.jpart && o.values && (y % o.stride) == 0)
        o.jpart[((size_t)b * o.n_times + o.slot) * o.M + y / o.stride] = 0.5 * s;
}

// A workgroup holds `tpb` teams; the launcher guarantees tpb divides the
// teams per member, so the member index is uniform over the workgroup and
// member base pointers live in scalar registers (32-bit lane offsets).  A
// team of at most 64 threads lies within one wavefront (WL): its exchanges
// synchronise the wave only, and the one workgroup barrier is the twiddle
// staging.
#define PA_TEAM_SETUP(N, V, TEAMS_PER_MEMBER)                           \
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E;                 \
    constexpr bool WL = T <= 64 && 64 % T == 0;                         \
    extern __shared__ cd smem[];                                        \
    const int team = threadIdx.x / T, t = threadIdx.x % T;              \
    cd* lds = smem + team * lds_team<N>();                              \
    const int tpb_ = blockDim.x / T;                                    \
    cd* const tw_lds = smem + tpb_ * lds_team<N>();                     \
    const int g0 = blockIdx.x * tpb_;                                   \
    const int b = g0 / (TEAMS_PER_MEMBER);                              \
    const int w0 = g0 % (TEAMS_PER_MEMBER);                             \
    const int wi = w0 + team;

// ------------------------------------------------------------ row passes --

// physical rows (y0, y0+1) -> Y rows; team per row pair.
template <int N, int V>
__global__ void __launch_bounds__(256) row_r2c_kernel(Dims d, const double* __restrict__ in,
                                                      cd* __restrict__ out, const cd* __restrict__ tw_g) {
    PA_TEAM_SETUP(N, V, N / 2)
    const double* r0 = in + ((size_t)b * N + 2 * w0) * N;     // block base (uniform)
    const int ro = 2 * team * N;                               // this team's row pair
    cd z[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + T * m;
        z[m] = mk(r0[ro + x], r0[ro + N + x]);
    }
    const cd* twl = stage_twiddles<N, V>(tw_lds, tw_g);
    fft<N, V, false, WL>(z, t, lds, twl);
    cd* o0 = out + ((size_t)b * N + 2 * wi) * kx_pad<N>();
    split_store<N, V, WL>(z, t, lds, o0, o0 + kx_pad<N>());
}

// Y rows (y0, y0+1) -> physical rows.
template <int N, int V>
__global__ void __launch_bounds__(256) row_c2r_kernel(Dims d, const cd* __restrict__ in,
                                                      double* __restrict__ out, const cd* __restrict__ tw_g) {
    PA_TEAM_SETUP(N, V, N / 2)
    const cd* i0 = in + ((size_t)b * N + 2 * wi) * kx_pad<N>();
    cd z[E];
    herm_load<N, V>(z, i0, i0 + kx_pad<N>(), t);
    const cd* twl = stage_twiddles<N, V>(tw_lds, tw_g);
    fft<N, V, true, WL>(z, t, lds, twl);
    double* r0 = out + ((size_t)b * N + 2 * w0) * N;
    const int ro = 2 * team * N;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + T * m;
        r0[ro + x] = z[m].x;
        r0[ro + N + x] = z[m].y;
    }
}

// Right-hand side products of one row:  q = u w_x + v w_y.  Inputs
// yin[0..3] = the packed pairs (u, w_x) P, Q and (v, w_y) P, Q of the stage,
// output yout[0] = row transform of q.
// Every input load is issued before the first transform, so the memory
// latency is paid once per kernel rather than once per transform.
// Observations are formed by row_obs_kernel from the same fields.
template <int N, int V>
__device__ __forceinline__ void row_nl_body(const Dims& d, const RowArgs& a) {
    const cd* __restrict__ tw_g = a.tw;
    PA_TEAM_SETUP(N, V, N)
    const int y = wi;
    const size_t roff = ((size_t)b * N + y) * kx_pad<N>();
    cd z1[E], z2[E];
    packed_load<N, V>(z1, a.yin[0] + roff, a.yin[1] + roff, t);   // u + i w_x
    packed_load<N, V>(z2, a.yin[2] + roff, a.yin[3] + roff, t);   // v + i w_y
    RowTw<N, V> tr;   // the three transforms of the row share the thread's twiddles
    row_twiddles<N, V>(tr, t, tw_g, tw_lds);
    row_fft<N, V, true, WL>(z1, t, lds, tr);
    row_fft<N, V, true, WL>(z2, t, lds, tr);
    cd z[E];
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = mk(z1[m].x * z1[m].y + z2[m].x * z2[m].y, 0.0);
    row_fft<N, V, false, WL>(z, t, lds, tr);
    cd* o = a.yout[0] + roff;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + T * m;
        if (slot_low<N, V>(m) && k <= band<N>()) o[k] = z[m];
    }
}

// Occupancy hint for the right-hand-side row pass: three waves per SIMD (168
// VGPRs).  With 8 register slots per thread (one row per team) the row's data
// and its twiddle factors in registers fit; at four waves (128 VGPRs) the
// twiddles spill, and reading them from LDS instead is 3.5 % slower at 256^2.
// The two-row kernel of the 4-slot plan holds both rows' loads.
template <int N, int V>
constexpr int nl_waves() { return Plan<N, V>::E <= 8 ? 3 : 1; }

// Two rows per team: q of both rows is real, so one complex transform of
// q_a + i q_b, split into the two half spectra, replaces two transforms of
// real signals (2.5 transforms per row instead of 3).  Used with the
// four-values-per-thread plan, where both rows' signals fit in registers.
template <int N, int V>
__device__ __forceinline__ void row_nl_pair_body(const Dims& d, const RowArgs& a) {
    const cd* __restrict__ tw_g = a.tw;
    PA_TEAM_SETUP(N, V, N / 2)
    constexpr int KXP = kx_pad<N>();
    const size_t ra = ((size_t)b * N + 2 * wi) * KXP, rb = ra + KXP;
    cd z1[E], z2[E], y1[E], y2[E];
    packed_load<N, V>(z1, a.yin[0] + ra, a.yin[1] + ra, t);   // row a: u + i w_x
    packed_load<N, V>(z2, a.yin[2] + ra, a.yin[3] + ra, t);   //        v + i w_y
    packed_load<N, V>(y1, a.yin[0] + rb, a.yin[1] + rb, t);   // row b
    packed_load<N, V>(y2, a.yin[2] + rb, a.yin[3] + rb, t);
    cd z[E];
    if constexpr (wave256<N, V>()) {
        RowTw<N, V> tr;
        row_twiddles<N, V>(tr, t, tw_g, tw_lds);
        row_fft<N, V, true, WL>(z1, t, lds, tr);
        row_fft<N, V, true, WL>(z2, t, lds, tr);
        row_fft<N, V, true, WL>(y1, t, lds, tr);
        row_fft<N, V, true, WL>(y2, t, lds, tr);
#pragma unroll
        for (int m = 0; m < E; ++m)
            z[m] = mk(z1[m].x * z1[m].y + z2[m].x * z2[m].y, y1[m].x * y1[m].y + y2[m].x * y2[m].y);
        row_fft<N, V, false, WL>(z, t, lds, tr);
    } else {
        const cd* twl = stage_twiddles<N, V>(tw_lds, tw_g);
        fft<N, V, true, WL>(z1, t, lds, twl);
        fft<N, V, true, WL>(z2, t, lds, twl);
        fft<N, V, true, WL>(y1, t, lds, twl);
        fft<N, V, true, WL>(y2, t, lds, twl);
#pragma unroll
        for (int m = 0; m < E; ++m)
            z[m] = mk(z1[m].x * z1[m].y + z2[m].x * z2[m].y, y1[m].x * y1[m].y + y2[m].x * y2[m].y);
        fft<N, V, false, WL>(z, t, lds, twl);
    }
    split_store<N, V, WL>(z, t, lds, a.yout[0] + ra, a.yout[0] + rb);
}

// Variant 2 runs two rows per team where its plan has four values per thread
// (16 to 256 points); with eight values the two rows' signals spill.
template <int N>
__host__ __device__ constexpr bool nl_pairs() { return Plan<N, 2>::E == 4; }

template <int N, int V>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(nl_waves<N, V>())))
row_nl_kernel(Dims d, RowArgs a) {
    if constexpr (V == 2 && nl_pairs<N>()) row_nl_pair_body<N, V>(d, a);
    else row_nl_body<N, V>(d, a);
}

// Observation of one step: team per observed row; yin[0..3] = the stage's
// packed pairs (u, w_x) and (v, w_y); u and v are the real parts of their row
// transforms.
template <int N, int V>
__global__ void __launch_bounds__(256) row_obs_kernel(Dims d, RowArgs a) {
    const cd* __restrict__ tw_g = a.tw;
    PA_TEAM_SETUP(N, V, a.obs.M)
    const int y = wi * a.obs.stride;
    const size_t roff = ((size_t)b * N + y) * kx_pad<N>();
    cd z1[E], z2[E];
    packed_load<N, V>(z1, a.yin[0] + roff, a.yin[1] + roff, t);
    packed_load<N, V>(z2, a.yin[2] + roff, a.yin[3] + roff, t);
    const cd* twl = stage_twiddles<N, V>(tw_lds, tw_g);
    fft<N, V, true, WL>(z1, t, lds, twl);
    fft<N, V, true, WL>(z2, t, lds, twl);
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        part += observe_comp(a.obs, b, y, t + T * m, 0, z1[m].x);
        part += observe_comp(a.obs, b, y, t + T * m, 1, z2[m].x);
    }
    const double s = team_sum<N, V, WL>(part, t, lds);
    if (t == 0) store_jpart(a.obs, b, y, s);
}

// Occupancy hint for the adjoint row pass: with 8 register slots per thread
// its three input signals fit the 168 VGPRs of three waves per SIMD (a couple
// of spilled values at most); with 16 slots the hint would spill heavily.
template <int N, int V>
constexpr int adj_waves() { return Plan<N, V>::E <= 8 ? 3 : 1; }

// The 1024-point plans of eight values per thread (two wavefronts per row)
// read their twiddles from the LDS table in the adjoint rows: their 19
// register factors would spill 64 values per thread at three waves per SIMD,
// and from LDS the kernel fits in 162 VGPRs.  Measured at 1024^2 with four
// and eight members: 69.0 -> 55.0 and 131 -> 96 us per launch.  The forward
// rows keep register twiddles (there LDS is 6-7 % slower).
template <int N, int V>
constexpr bool adj_tw_lds() { return (N == 1024 || N == 512) && Plan<N, V>::E == 8; }

// Adjoint products of one row.  The transpose of the tangent right-hand side
// applied to lambda, with Lam = P lambda, is on the de-aliased band
//   (1/|k|^2) F[w_x Lam_y - w_y Lam_x] + F[u Lam_x + v Lam_y]
// (the product rule holds on the band because the 2/3 rule keeps every alias
// outside it, and u_x + v_y = 0).  Inputs yin[0..3] = the packed pairs (u, w_x)
// and (v, w_y) of the stage state, yin[4..5] = the packed pair (Lam_x, Lam_y).
// Outputs: the row transform Z of G1 + i G2, G1 = w_x Lam_y - w_y Lam_x and
// G2 = u Lam_x + v Lam_y, unsplit (pair_store): yout[0] = Z, yout[1] = conj Z(-k).
template <int N, int V>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(adj_waves<N, V>())))
row_adj_kernel(Dims d, RowArgs a) {
    const cd* __restrict__ tw_g = a.tw;
    PA_TEAM_SETUP(N, V, N)
    const int y = wi;
    const size_t roff = ((size_t)b * N + y) * kx_pad<N>();
    cd L[E], z1[E], z2[E];   // (Lam_x, Lam_y), (u, w_x), (v, w_y)
    packed_load<N, V>(L, a.yin[4] + roff, a.yin[5] + roff, t);
    packed_load<N, V>(z1, a.yin[0] + roff, a.yin[1] + roff, t);
    packed_load<N, V>(z2, a.yin[2] + roff, a.yin[3] + roff, t);
    cd G[E];   // (G1, G2)
    auto products = [&]() {
#pragma unroll
        for (int m = 0; m < E; ++m)
            G[m] = mk(z1[m].y * L[m].y - z2[m].y * L[m].x, z1[m].x * L[m].x + z2[m].x * L[m].y);
    };
    if constexpr (adj_tw_lds<N, V>()) {
        const cd* twl = stage_twiddles<N, V>(tw_lds, tw_g);
        fft<N, V, true, WL>(L, t, lds, twl);
        fft<N, V, true, WL>(z1, t, lds, twl);
        fft<N, V, true, WL>(z2, t, lds, twl);
        products();
        fft<N, V, false, WL>(G, t, lds, twl);
    } else {
        RowTw<N, V> tr;   // the four transforms of the row share the thread's twiddles
        row_twiddles<N, V>(tr, t, tw_g, tw_lds);
        row_fft<N, V, true, WL>(L, t, lds, tr);
        row_fft<N, V, true, WL>(z1, t, lds, tr);
        row_fft<N, V, true, WL>(z2, t, lds, tr);
        products();
        row_fft<N, V, false, WL>(G, t, lds, tr);
    }
    pair_store<N, V>(G, t, a.yout[0] + roff, a.yout[1] + roff);
}

// Adjoint source rows.  mode 0: observation residual at one observed step
// (yin[0..3] = the packed pairs (u, w_x), (v, w_y) of that state); mode 1:
// unit u-impulse at (imp_x, imp_y).
// Outputs yout[0] = row transform of -S^T r_u, yout[1] = of -S^T r_v.
template <int N, int V>
__global__ void __launch_bounds__(256) row_src_kernel(Dims d, RowArgs a, int impulse) {
    const cd* __restrict__ tw_g = a.tw;
    PA_TEAM_SETUP(N, V, N)
    const int y = wi;
    const size_t roff = ((size_t)b * N + y) * kx_pad<N>();
    const RowObs& o = a.obs;
    cd z[E], z2[E];
    if (!impulse) {
        packed_load<N, V>(z, a.yin[0] + roff, a.yin[1] + roff, t);
        packed_load<N, V>(z2, a.yin[2] + roff, a.yin[3] + roff, t);
    }
    const cd* twl = stage_twiddles<N, V>(tw_lds, tw_g);
    if (!impulse) {
        fft<N, V, true, WL>(z, t, lds, twl);
        fft<N, V, true, WL>(z2, t, lds, twl);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + T * m;
        double A = 0.0, Bv = 0.0;
        if (impulse) {
            if (x == o.imp_x && y == o.imp_y) A = -1.0;
        } else if (o.values && (y % o.stride) == 0 && (x % o.stride) == 0) {
            const int i = x / o.stride, j = y / o.stride, M = o.M;
            const size_t base = (((size_t)b * o.n_times + o.slot) * 2) * M * M + (size_t)j * M + i;
            A = -(z[m].x - o.values[base]);
            Bv = -(z2[m].x - o.values[base + (size_t)M * M]);
        }
        z[m] = mk(A, Bv);
    }
    fft<N, V, false, WL>(z, t, lds, twl);
    split_store<N, V, WL>(z, t, lds, a.yout[0] + roff, a.yout[1] + roff);
}

// ---------------------------------------------------------- column pass --

__device__ __forceinline__ int band_row(int q, int N, int K, int KY) {
    if (q <= K) return q;
    if (q >= N - K) return q - N + KY;
    return -1;
}

// Position of workgroup `id` of a one-dimensional grid of `n` in an order in
// which each XCD holds a contiguous run: workgroup id runs on XCD id % XCDS
// (round-robin dispatch), and that XCD's k-th workgroup takes the k-th entry
// of its run.  A bijection of 0..n-1 for any n, so only locality depends on it.
constexpr unsigned XCDS = 8;
__device__ __forceinline__ unsigned xcd_order(unsigned id, unsigned n) {
    const unsigned x = id % XCDS, k = id / XCDS;
    const unsigned q = n / XCDS, r = n % XCDS;   // XCDs below r hold q + 1 workgroups
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Occupancy hint for the column pass: three waves per SIMD (168 VGPRs) for the
// plans of up to eight values per thread; sixteen values per thread are left
// unconstrained (a cap there spills hundreds of bytes).
template <int N, int V>
constexpr int col_waves() { return Plan<N, V>::E <= 8 ? 3 : 1; }

// Up to 512 threads: CB columns of T threads each (CB * T <= 512).
template <int N, int V, int MODE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(col_waves<N, V>()))) col_kernel(Dims d, ColArgs a) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E;
    constexpr bool FWD_STAGE = MODE >= COL_A && MODE <= COL_D;
    constexpr bool ADJ = (MODE >= COL_ADJ_C && MODE <= COL_ADJ_SRC) || MODE == COL_ADJ_NSRC;
    constexpr bool STAGE_N = MODE == COL_ADJ_N || MODE == COL_ADJ_NSRC;
    extern __shared__ cd smem[];
    const int CB = d.cb;
    const int c = threadIdx.x % CB, t = threadIdx.x / CB;
    cd* lds = smem + c * lds_team<N>();
    // One-dimensional grid of (member, column block, share) in that order,
    // share fastest.  The hardware hands workgroups to the XCDs round robin by
    // id; each XCD is given a contiguous run of that order instead, so that the
    // column blocks of one 128-byte line and the shares of one column meet in
    // one L2 rather than fetching and writing the line from several.
    const unsigned wg = xcd_order(blockIdx.x, gridDim.x);
    const int zs = (int)(wg % (unsigned)a.split);   // share of the derived fields
    const unsigned cbk = wg / (unsigned)a.split;
    const unsigned nblk = (unsigned)(d.KXP / CB);
    const int b = (int)(cbk / nblk);
    const bool writer = zs == 0;               // the share that writes the compact outputs
    const int kx0 = (int)(cbk % nblk) * CB;    // uniform first column of the block
    const int kx = kx0 + c;
    constexpr int K = band<N>(), KXP = kx_pad<N>(), KY = 2 * K + 1;
    const bool colok = kx <= K;
    // uniform bases (scalar registers) + 32-bit lane offsets
    const size_t ymem = (size_t)b * N * KXP + kx0;
    const size_t cmem = (size_t)b * KY * KXP + kx0;
    const unsigned ylane = (unsigned)c;         // + y * KXP
    const double* __restrict__ ik2t = a.invk2 + kx0;
    const double dkx = (double)kx;
    const double ex = a.ex2[kx];
    const double h = a.h;
    auto yoff = [&](int m) { return ylane + (unsigned)(t + T * m) * (unsigned)KXP; };
    // compact row of slot m, -1 off the band (gap slots fold to -1 at compile time)
    auto rowof = [&](int m) { return (slot_in_band<N, V>(m) && colok) ? band_row(t + T * m, N, K, KY) : -1; };
    auto inS = [&](int r) { return r >= 0 && !(kx == 0 && r == 0); };
    auto cidx = [&](int r) { return (unsigned)c + (unsigned)r * (unsigned)KXP; };

    // ---- issue every global load first: input column(s) and compact operands.
    // Loads are unconditional at in-bounds addresses (padding columns kx < KXP,
    // compact row 0 for rows off the band) and their results selected, so no
    // load sits in a branch.
    cd v0[E];          // first input column
    cd v1[E];          // second input column (adjoint)
    cd s0[E], s1[E];   // compact operands: (omega_n, acc) forward, (lambda, omega-bar) adjoint
    if constexpr (MODE != COL_FROM_STATE) {
        const cd* __restrict__ src = a.yin[0] + ymem;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const cd x = ldc(src, yoff(m));
            v0[m] = colok ? x : czero();
        }
    }
    if constexpr (ADJ || MODE == COL_FIRST_GUESS) {
        const cd* __restrict__ src = a.yin[1] + ymem;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const cd x = ldc(src, yoff(m));
            v1[m] = colok ? x : czero();
        }
    }
    // compact operands; the adjoint modes issue them after their first input
    // transform, which keeps two input columns, the accumulator and these
    // operands from being live at once (the registers set the occupancy)
    const bool need1 = (FWD_STAGE && MODE != COL_A) || (ADJ && MODE != COL_ADJ_C && MODE != COL_ADJ_SRC);
    const bool need0 = !(ADJ && (STAGE_N || MODE == COL_ADJ_SRC));
    auto load_compact = [&](bool do0, bool do1) {
        const cd* __restrict__ p0 = FWD_STAGE ? a.omega + cmem : ADJ ? a.lam + cmem : a.state_in + cmem;
        const cd* __restrict__ p1 = FWD_STAGE ? a.acc + cmem : (ADJ && MODE != COL_ADJ_SRC) ? a.omb + cmem : nullptr;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (do0) s0[m] = czero();
            if (do1) s1[m] = czero();
            if (!slot_in_band<N, V>(m)) continue;
            const int r = rowof(m);
            const unsigned ci = cidx(r >= 0 ? r : 0);
            if (do0 && need0) {
                const cd x = ldc(p0, ci);
                s0[m] = r >= 0 ? x : czero();
            }
            if (do1 && need1) {
                const cd x = ldc(p1, ci);
                s1[m] = r >= 0 ? x : czero();
            }
        }
    };
    if constexpr (FWD_STAGE || MODE == COL_FROM_STATE) load_compact(true, true);
    const cd* twl = stage_twiddles<N, V>(smem + CB * lds_team<N>(), a.tw);

    cd w[E];   // spectral values handed to the output transforms

    if constexpr (MODE <= COL_FILTER) {
        fft<N, V, false>(v0, t, lds, twl);
        cd* __restrict__ om = (writer && a.omega) ? (MODE == COL_D && a.omega_out ? a.omega_out : a.omega) + cmem
                                                  : nullptr;
        cd* __restrict__ ac = (writer && a.acc) ? a.acc + cmem : nullptr;
        cd* __restrict__ ck = (writer && a.ckpt) ? a.ckpt + cmem : nullptr;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rowof(m);
            if (r < 0) { w[m] = czero(); continue; }
            const unsigned ci = cidx(r);
            const bool ins = inS(r);
            if constexpr (MODE == COL_INIT) {
                const cd s = ins ? v0[m] : czero();
                if (om) stc(om, ci, s);
                if (ck) stc(ck, ci, s);
                w[m] = s;
            } else if constexpr (MODE == COL_FILTER) {
                const size_t mi = (a.mult_per_member ? (size_t)b * KY * KXP : 0) + (size_t)r * KXP + kx;
                w[m] = ins ? cscale(v0[m], a.mult[mi]) : czero();
            } else {
                const int ky = (r <= K) ? r : r - KY;
                cd nl = ins ? mk(-v0[m].x, -v0[m].y) : czero();
                if (a.nf > 0 && kx == 0 && (ky == a.nf || ky == -a.nf)) nl.x += a.forcing;
                const double e2 = ex * a.ey2[r];
                const double e1 = e2 * e2;
                const cd wn = s0[m];
                if constexpr (MODE == COL_A) {
                    if (ac) stc(ac, ci, cscale(nl, e1));
                    w[m] = cscale(mk(wn.x + 0.5 * h * nl.x, wn.y + 0.5 * h * nl.y), e2);
                } else if constexpr (MODE == COL_B) {
                    const cd q = s1[m];
                    if (ac) stc(ac, ci, mk(q.x + 2.0 * e2 * nl.x, q.y + 2.0 * e2 * nl.y));
                    w[m] = mk(e2 * wn.x + 0.5 * h * nl.x, e2 * wn.y + 0.5 * h * nl.y);
                } else if constexpr (MODE == COL_C) {
                    const cd q = s1[m];
                    if (ac) stc(ac, ci, mk(q.x + 2.0 * e2 * nl.x, q.y + 2.0 * e2 * nl.y));
                    w[m] = mk(e1 * wn.x + h * e2 * nl.x, e1 * wn.y + h * e2 * nl.y);
                } else {   // COL_D
                    const cd q = s1[m];
                    const double h6 = h / 6.0;
                    const cd s = mk(e1 * wn.x + h6 * (q.x + nl.x), e1 * wn.y + h6 * (q.y + nl.y));
                    if (om) stc(om, ci, s);
                    if (ck) stc(ck, ci, s);
                    w[m] = s;
                }
            }
        }
    } else if constexpr (MODE == COL_FIRST_GUESS) {
        // vorticity of the low-passed probe velocity: i kx v_hat - i ky u_hat on S
        fft<N, V, false>(v0, t, lds, twl);
        fft<N, V, false>(v1, t, lds, twl);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rowof(m);
            const int ky = (r <= K) ? r : r - KY;
            const bool keep = inS(r) && kx <= a.lowpass && ky <= a.lowpass && -ky <= a.lowpass;
            w[m] = keep ? mk(-dkx * v1[m].y + (double)ky * v0[m].y, dkx * v1[m].x - (double)ky * v0[m].x) : czero();
        }
    } else if constexpr (MODE == COL_FROM_STATE) {
        cd* __restrict__ om = (writer && a.omega) ? a.omega + cmem : nullptr;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rowof(m);
            if (r < 0) { w[m] = czero(); continue; }
            const cd s = inS(r) ? s0[m] : czero();
            if (om) stc(om, cidx(r), s);
            w[m] = s;
        }
    } else {
        // adjoint: wbar = 1_S sum_p mult_p F_y(yin[p]), mult_p selected by inmul[p]
        auto accumulate = [&](cd* v, int mk_) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int r = rowof(m);
                if (!inS(r)) continue;
                const double ky = (double)((r <= K) ? r : r - KY);
                const double ik2 = ik2t[cidx(r)];
                if (mk_ == IN_PAIRP) {          // v (1/|k|^2 - i) / 2
                    w[m].x += 0.5 * (ik2 * v[m].x + v[m].y);
                    w[m].y += 0.5 * (ik2 * v[m].y - v[m].x);
                } else if (mk_ == IN_PAIRQ) {   // v (1/|k|^2 + i) / 2
                    w[m].x += 0.5 * (ik2 * v[m].x - v[m].y);
                    w[m].y += 0.5 * (ik2 * v[m].y + v[m].x);
                } else {
                    const double f = (mk_ == IN_IKY_INVK2) ? ky * ik2 : -dkx * ik2;   // i f v
                    w[m].x -= f * v[m].y;
                    w[m].y += f * v[m].x;
                }
            }
        };
#pragma unroll
        for (int m = 0; m < E; ++m) w[m] = czero();
        fft<N, V, false>(v0, t, lds, twl);
        accumulate(v0, a.inmul[0]);
        // compact operands in flight during the second input transform: a
        // stage's only one, or of two (B and A) lambda, up to 256 points; from
        // 512 points the pair is issued after it (lambda live through the
        // transform spills there under the three-wave cap)
        const bool both = need0 && need1;
        if (!both || N <= 256) load_compact(true, !both);
        fft<N, V, false>(v1, t, lds, twl);
        accumulate(v1, a.inmul[1]);
        if (both) load_compact(N > 256, true);
        // observation sources enter at stage n of an observed step only (two more inputs)
        if constexpr (MODE == COL_ADJ_NSRC)
        for (int p = 2; p < a.nin; ++p) {
            const cd* __restrict__ src = a.yin[p] + ymem;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const cd x = ldc(src, yoff(m));
                v0[m] = colok ? x : czero();
            }
            fft<N, V, false>(v0, t, lds, twl);
            accumulate(v0, a.inmul[p]);
        }
        const double sc = a.scale ? a.scale[b] : 1.0;
        cd* __restrict__ lm_p = writer ? a.lam + cmem : nullptr;
        cd* __restrict__ ob_p = (writer && a.omb) ? a.omb + cmem : nullptr;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rowof(m);
            if (r < 0) { w[m] = czero(); continue; }
            const unsigned ci = cidx(r);
            const cd wb = w[m];   // zero off the band by construction
            const double e2 = ex * a.ey2[r];
            const double e1 = e2 * e2;
            if constexpr (MODE == COL_ADJ_C) {
                const cd lm = s0[m];
                if (ob_p) stc(ob_p, ci, mk(e1 * (lm.x + wb.x), e1 * (lm.y + wb.y)));
                w[m] = mk((h / 3.0) * e2 * lm.x + h * e2 * wb.x, (h / 3.0) * e2 * lm.y + h * e2 * wb.y);
            } else if constexpr (MODE == COL_ADJ_B) {
                const cd lm = s0[m], ob = s1[m];
                if (ob_p) stc(ob_p, ci, mk(ob.x + e2 * wb.x, ob.y + e2 * wb.y));
                w[m] = mk((h / 3.0) * e2 * lm.x + 0.5 * h * wb.x, (h / 3.0) * e2 * lm.y + 0.5 * h * wb.y);
            } else if constexpr (MODE == COL_ADJ_A) {
                const cd lm = s0[m], ob = s1[m];
                if (ob_p) stc(ob_p, ci, mk(ob.x + e2 * wb.x, ob.y + e2 * wb.y));
                w[m] = mk((h / 6.0) * e1 * lm.x + 0.5 * h * e2 * wb.x, (h / 6.0) * e1 * lm.y + 0.5 * h * e2 * wb.y);
            } else {   // stage n (with or without sources), COL_ADJ_SRC
                cd ln = wb;
                if constexpr (STAGE_N) {
                    const cd ob = s1[m];
                    ln = mk(ob.x + wb.x, ob.y + wb.y);
                }
                if (lm_p) stc(lm_p, ci, ln);
                w[m] = a.final_out ? cscale(ln, sc) : cscale(ln, h / 6.0);
            }
        }
    }

    // derived fields: 1_S * multiplier * w / N^2, inverse transform along y; a
    // packed pair half A +- i B is formed from the two multipliers before the
    // transform (the transform is linear)
    const double inv_n2 = 1.0 / ((double)N * (double)N);
    for (int o = zs; o < a.nout; o += a.split) {
        const int f = a.fields[o];
        cd v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rowof(m);
            if (!inS(r)) { v[m] = czero(); continue; }
            const double ky = (double)((r <= K) ? r : r - KY);
            const cd s = cscale(w[m], inv_n2);
            const double ik2 = ik2t[(unsigned)c + (unsigned)r * (unsigned)KXP];
            if (f == F_OMEGA) {
                v[m] = s;
            } else {
                cd A, Bf;
                if (f == F_UP || f == F_UQ) {          // (u, w_x) = (i ky / k^2, i kx) s
                    A = cscale(mul_i(s), ky * ik2);
                    Bf = cscale(mul_i(s), dkx);
                } else if (f == F_VP || f == F_VQ) {   // (v, w_y) = (-i kx / k^2, i ky) s
                    A = cscale(mul_i(s), -dkx * ik2);
                    Bf = cscale(mul_i(s), ky);
                } else {                               // (Lam_x, Lam_y) = (i kx, i ky) s
                    A = cscale(mul_i(s), dkx);
                    Bf = cscale(mul_i(s), ky);
                }
                const bool plus = f == F_UP || f == F_VP || f == F_LP;
                v[m] = plus ? mk(A.x - Bf.y, A.y + Bf.x) : mk(A.x + Bf.y, A.y - Bf.x);
            }
        }
        fft<N, V, true>(v, t, lds, twl);
        if (colok) {
            cd* __restrict__ out = a.yout[o] + ymem;
#pragma unroll
            for (int m = 0; m < E; ++m) stc(out, yoff(m), v[m]);
        }
    }
}

// ---------------------------------------- pipelined row passes (gfx950) --
// Variant 3 of the row passes: the plan of variant 2 run by persistent
// wavefronts.  A wavefront owns G = 64 / T consecutive rows of one member
// (contiguous in the Y layout) at a time and loops over such row groups.
// The half spectra of its next group stream from HBM straight into a
// per-wave LDS stage buffer (global->LDS loads: no registers are held while
// they are in flight) while it transforms the current group.  They are read
// into registers, with the Hermitian extension, just before the current
// group's outputs are stored, so the wait for them never waits on fresh
// stores.  Only the twiddle staging synchronises the workgroup.

constexpr int PIPE_V = 2;   // plan variant run by the pipelined kernels

template <int N>
struct Pipe {
    static constexpr int T = Plan<N, PIPE_V>::T, E = Plan<N, PIPE_V>::E;
    static constexpr int G = (T <= 64 && 64 % T == 0) ? 64 / T : 1;   // rows per wavefront
    static constexpr bool OK = T <= 64 && 64 % T == 0 && G <= N;
    static constexpr int KXP = kx_pad<N>();
    static constexpr int SPAN = G * KXP;                   // elements of one field of a row group
    static constexpr int LOADS = (SPAN + 63) / 64;         // 64-lane loads per field
    template <int NF>
    static constexpr int wave_lds() { return NF * SPAN + G * lds_team<N>(); }
    static __host__ __device__ size_t offset(int group) {  // first element of a row group
        constexpr int GPM = N / G;
        return ((size_t)(group / GPM) * N + (size_t)(group % GPM) * G) * KXP;
    }
};

__device__ __forceinline__ void vm_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Returns v unchanged, opaquely: index arithmetic derived from it inside a
// loop is not hoisted out of the loop (where its results would occupy
// registers for the loop's whole lifetime) but recomputed per iteration.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Global->LDS loads of one row group of NF fields into the wave's stage
// buffer (lane l of a load lands at the load's LDS base + l).  The LDS base
// of these loads goes to M0 and must be uniform over the wavefront: the
// full-wave loads are issued first with no condition, and the partial final
// loads of all fields together in one conditional block, so that the compiler
// never merges a masked load with a load of another LDS base (the merged
// instruction would take one lane's base for every lane).
template <int N, int NF>
__device__ __forceinline__ void pipe_fetch(cd* stage, const cd* const (&src)[NF], size_t off, int lane) {
    using P = Pipe<N>;
    constexpr int FULL = P::SPAN / 64, TAIL = P::SPAN % 64;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < FULL; ++i)
            __builtin_amdgcn_global_load_lds(src[f] + off + i * 64 + lane,
                                             (__attribute__((address_space(3))) void*)(stage + f * P::SPAN + i * 64),
                                             16, 0, 0);
    if constexpr (TAIL > 0) {
        if (lane < TAIL) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                __builtin_amdgcn_global_load_lds(src[f] + off + FULL * 64 + lane,
                                                 (__attribute__((address_space(3))) void*)(stage + f * P::SPAN + FULL * 64),
                                                 16, 0, 0);
        }
    }
}

template <int N>
__global__ void __launch_bounds__(256) row_nl_pipe_kernel(Dims d, RowArgs a, int n_groups) {
    using P = Pipe<N>;
    constexpr int V = PIPE_V, T = P::T, E = P::E, KXP = P::KXP, NF = 4, WL_ = true;
    extern __shared__ cd smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, team = lane / T, t0 = lane % T;
    const int wpg = blockDim.x >> 6;
    cd* const stage = smem + wave * P::template wave_lds<NF>();
    cd* const lds = stage + NF * P::SPAN + team * lds_team<N>();
    RowTw<N, V> tr;
    row_twiddles<N, V>(tr, t0, a.tw, smem + wpg * P::template wave_lds<NF>());
    const int nw = gridDim.x * wpg;
    int g = blockIdx.x * wpg + wave;
    const cd* const src[NF] = {a.yin[0], a.yin[1], a.yin[2], a.yin[3]};   // packed (u, w_x), (v, w_y)
    const cd* const row = stage + team * KXP;
    cd z1[E], z2[E];
    if (g < n_groups) {
        pipe_fetch<N, NF>(stage, src, P::offset(g), lane);
        vm_wait();
        packed_load<N, V>(z1, row, row + P::SPAN, t0);
        wave_lds_sync();
        packed_load<N, V>(z2, row + 2 * P::SPAN, row + 3 * P::SPAN, t0);
        wave_lds_sync();
        if (g + nw < n_groups) pipe_fetch<N, NF>(stage, src, P::offset(g + nw), lane);
    }
    for (; g < n_groups; g += nw) {
        const int t = opaque(t0);
        row_fft<N, V, true, WL_>(z1, t, lds, tr);
        row_fft<N, V, true, WL_>(z2, t, lds, tr);
        cd z[E];
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = mk(z1[m].x * z1[m].y + z2[m].x * z2[m].y, 0.0);
        row_fft<N, V, false, WL_>(z, t, lds, tr);
        const int gn = g + nw;
        if (gn < n_groups) {
            vm_wait();
            packed_load<N, V>(z1, row, row + P::SPAN, t);
            wave_lds_sync();
            packed_load<N, V>(z2, row + 2 * P::SPAN, row + 3 * P::SPAN, t);
            wave_lds_sync();
            if (gn + nw < n_groups) pipe_fetch<N, NF>(stage, src, P::offset(gn + nw), lane);
        }
        cd* o = a.yout[0] + P::offset(g) + team * KXP;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int k = t + T * m;
            if (slot_low<N, V>(m) && k <= band<N>()) o[k] = z[m];
        }
    }
}

template <int N>
__global__ void __launch_bounds__(256) row_adj_pipe_kernel(Dims d, RowArgs a, int n_groups) {
    using P = Pipe<N>;
    constexpr int V = PIPE_V, T = P::T, E = P::E, KXP = P::KXP, NF = 6, WL_ = true;
    extern __shared__ cd smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, team = lane / T, t0 = lane % T;
    const int wpg = blockDim.x >> 6;
    cd* const stage = smem + wave * P::template wave_lds<NF>();
    cd* const lds = stage + NF * P::SPAN + team * lds_team<N>();
    RowTw<N, V> tr;
    row_twiddles<N, V>(tr, t0, a.tw, smem + wpg * P::template wave_lds<NF>());
    const int nw = gridDim.x * wpg;
    int g = blockIdx.x * wpg + wave;
    // packed (Lam_x, Lam_y), (u, w_x), (v, w_y)
    const cd* const src[NF] = {a.yin[4], a.yin[5], a.yin[0], a.yin[1], a.yin[2], a.yin[3]};
    const cd* const row = stage + team * KXP;
    cd L[E], z1[E], z2[E];
    // one signal pair at a time: LDS latency is short, and the raw values of
    // all three pairs in flight at once would double the registers held
    auto read_inputs = [&](int t) {
        packed_load<N, V>(L, row, row + P::SPAN, t);
        wave_lds_sync();
        packed_load<N, V>(z1, row + 2 * P::SPAN, row + 3 * P::SPAN, t);
        wave_lds_sync();
        packed_load<N, V>(z2, row + 4 * P::SPAN, row + 5 * P::SPAN, t);
        wave_lds_sync();
    };
    if (g < n_groups) {
        pipe_fetch<N, NF>(stage, src, P::offset(g), lane);
        vm_wait();
        read_inputs(t0);
        if (g + nw < n_groups) pipe_fetch<N, NF>(stage, src, P::offset(g + nw), lane);
    }
    for (; g < n_groups; g += nw) {
        const int t = opaque(t0);
        row_fft<N, V, true, WL_>(L, t, lds, tr);
        row_fft<N, V, true, WL_>(z1, t, lds, tr);
        row_fft<N, V, true, WL_>(z2, t, lds, tr);
        cd G[E];
#pragma unroll
        for (int m = 0; m < E; ++m)
            G[m] = mk(z1[m].y * L[m].y - z2[m].y * L[m].x, z1[m].x * L[m].x + z2[m].x * L[m].y);
        row_fft<N, V, false, WL_>(G, t, lds, tr);
        const int gn = g + nw;
        if (gn < n_groups) {
            vm_wait();
            read_inputs(t);
            if (gn + nw < n_groups) pipe_fetch<N, NF>(stage, src, P::offset(gn + nw), lane);
        }
        const size_t ro = P::offset(g) + team * KXP;
        pair_store<N, V>(G, t, a.yout[0] + ro, a.yout[1] + ro);
    }
}

// Persistent grid: as many workgroups as can be resident (occupancy query,
// cached per kernel and workgroup size), at most one row group per wave.
template <int N, int NF, class Kern>
hipError_t pipe_launch(Kern kernel, int teams, const Dims& d, const RowArgs& a, hipStream_t s) {
    using P = Pipe<N>;
    const int n_groups = d.B * (N / P::G);
    const int wpg = teams >= 4 ? 4 : teams >= 2 ? 2 : 1;
    const size_t lds = ((size_t)wpg * P::template wave_lds<NF>() + N) * sizeof(cd);
    static std::atomic<int> per_cu_cache[3];
    std::atomic<int>& slot = per_cu_cache[wpg == 1 ? 0 : wpg == 2 ? 1 : 2];
    int per_cu = slot.load(std::memory_order_relaxed);
    if (per_cu <= 0) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, wpg * 64, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) return hipErrorInvalidConfiguration;
        slot.store(per_cu, std::memory_order_relaxed);
    }
    const long want = (n_groups + wpg - 1) / wpg;
    const long wgs = std::min<long>(want, (long)per_cu * std::max(d.cus, 1));
    launch_kernel(kernel, dim3((unsigned)wgs), dim3((unsigned)(wpg * 64)), lds, s, d, a, n_groups);
    return hipGetLastError();
}

// ------------------------------------------------------------- launchers --

// Teams per workgroup: must divide the teams per member (the kernels take the
// member index from the workgroup's first team), fit 256 threads and 64 KiB
// of LDS.
template <int N, int V>
int row_tpb(int tpb, long teams_per_member) {
    const int cap = 256 / Plan<N, V>::T;
    if (tpb > cap) tpb = cap;
    if (tpb < 1) tpb = 1;
    while (tpb > 1 && ((size_t)tpb * lds_team<N>() + N) * sizeof(cd) > 65536) tpb >>= 1;
    while (tpb > 1 && teams_per_member % tpb) tpb >>= 1;
    return tpb;
}

template <int N, int V>
size_t row_lds(int tpb) { return ((size_t)tpb * lds_team<N>() + N) * sizeof(cd); }

#define PA_ROW_LAUNCH_V(V, TPB, KERNEL, ...)                                                   \
    do {                                                                                       \
        const int tpb = row_tpb<N, V>((TPB), tpm_);                                            \
        const dim3 grid_((unsigned)(teams_ / tpb));                                            \
        const dim3 block_((unsigned)(tpb * Plan<N, V>::T));                                    \
        const size_t lds_ = row_lds<N, V>(tpb);                                                \
        launch_kernel(KERNEL<N, V>, grid_, block_, lds_, s, __VA_ARGS__);                       \
    } while (0)

// VAR / TPB: the plan variant and rows per workgroup of the launching pass
// (forward rows: d.var, d.tpb; adjoint rows: d.avar, d.atpb).  Variant 3
// (pipelined) runs the plan of variant 2 in the kernels it does not cover.
#define PA_ROW_LAUNCH(VAR, TPB, KERNEL, TEAMS_PER_MEMBER, ...)                                 \
    do {                                                                                       \
        const long tpm_ = (TEAMS_PER_MEMBER);                                                  \
        const long teams_ = tpm_ * d.B;                                                        \
        if ((VAR) == 0) PA_ROW_LAUNCH_V(0, TPB, KERNEL, __VA_ARGS__);                          \
        else if ((VAR) == 1) PA_ROW_LAUNCH_V(1, TPB, KERNEL, __VA_ARGS__);                     \
        else PA_ROW_LAUNCH_V(2, TPB, KERNEL, __VA_ARGS__);                                     \
        return hipGetLastError();                                                              \
    } while (0)

template <int N>
hipError_t Launch<N>::row_r2c(const Dims& d, const double* in, cd* out, const cd* tw, hipStream_t s) {
    PA_ROW_LAUNCH(d.var, d.tpb, row_r2c_kernel, N / 2, d, in, out, tw);
}
template <int N>
hipError_t Launch<N>::row_c2r(const Dims& d, const cd* in, double* out, const cd* tw, hipStream_t s) {
    PA_ROW_LAUNCH(d.var, d.tpb, row_c2r_kernel, N / 2, d, in, out, tw);
}
template <int N>
hipError_t Launch<N>::row_nl(const Dims& d, const RowArgs& a, hipStream_t s) {
    // variant 3 without a pipelined kernel for N falls back to the variant-2 kernel launched with
    // one team per row below, which must then be the one-row kernel
    static_assert(Pipe<N>::OK || !nl_pairs<N>(), "the variant-3 fallback would launch the two-row kernel");
    if constexpr (Pipe<N>::OK)
        if (d.var == 3) return pipe_launch<N, 4>(row_nl_pipe_kernel<N>, d.tpb, d, a, s);
    if (d.var == 2 && nl_pairs<N>()) PA_ROW_LAUNCH(d.var, d.tpb, row_nl_kernel, N / 2, d, a);   // two rows per team
    PA_ROW_LAUNCH(d.var, d.tpb, row_nl_kernel, N, d, a);
}
template <int N>
hipError_t Launch<N>::row_obs(const Dims& d, const RowArgs& a, hipStream_t s) {
    PA_ROW_LAUNCH(d.var, d.tpb, row_obs_kernel, a.obs.M, d, a);
}
template <int N>
hipError_t Launch<N>::row_adj(const Dims& d, const RowArgs& a, hipStream_t s) {
    if constexpr (Pipe<N>::OK)
        if (d.avar == 3) return pipe_launch<N, 6>(row_adj_pipe_kernel<N>, d.atpb, d, a, s);
    PA_ROW_LAUNCH(d.avar, d.atpb, row_adj_kernel, N, d, a);
}
template <int N>
hipError_t Launch<N>::row_src(const Dims& d, const RowArgs& a, int impulse, hipStream_t s) {
    PA_ROW_LAUNCH(d.avar, d.atpb, row_src_kernel, N, d, a, impulse);
}

// Workgroups that share out one column's derived fields.  A launch whose
// columns cannot keep two wavefronts per SIMD busy (small batches of large
// grids: 1024^2 has 344 columns) is latency-bound by each column's chain of
// transforms; each share recomputes the input transform(s) and combine and
// runs its part of the output transforms, so the chain is shorter and more
// wavefronts are in flight.  The derived fields are the same whatever the
// split (each share runs the same operations), so results do not depend on it.
// d.csplit > 0 fixes the number of shares (capped at the output count);
// 0 picks 1, 2 or 4 from the wavefronts the launch has without a split.
template <int N, int V>
int col_split(const Dims& d, int nout) {
    if (nout <= 1) return 1;
    if (d.csplit > 0) return std::min(d.csplit, nout);
    const long waves = (long)(d.KXP / d.cb) * d.B * ((d.cb * Plan<N, V>::T + 63) / 64);
    const long target = 8L * std::max(d.cus, 1);   // two wavefronts per SIMD
    int split = 1;
    while (split < nout && waves * split < target) split *= 2;
    return std::min(split, nout);
}

template <int N, int V, int MODE>
hipError_t col_mode(const Dims& d, const ColArgs& a, hipStream_t s) {
    ColArgs ak = a;
    ak.split = col_split<N, V>(d, a.nout);
    const dim3 grid((unsigned)(d.KXP / d.cb) * (unsigned)d.B * (unsigned)ak.split);
    const dim3 block((unsigned)(d.cb * Plan<N, V>::T));
    const size_t lds = ((size_t)d.cb * lds_team<N>() + N) * sizeof(cd);
    // Column blocks wider than 64 KiB of LDS (1024-point columns, four or more
    // per workgroup): the kernel's dynamic LDS limit is raised to the
    // device's once per instantiation.  Such a block fills a CU alone, so it
    // pays only where a launch has few columns (one 1024^2 member: 25.1
    // against 26.8 us per forward stage); the autotuner decides.
    if (lds > 65536) {
        static const hipError_t raised = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&col_kernel<N, V, MODE>), hipFuncAttributeMaxDynamicSharedMemorySize,
            d.lds_max);
        if (raised != hipSuccess) return raised;
    }
    launch_kernel(col_kernel<N, V, MODE>, grid, block, lds, s, d, ak);
    return hipGetLastError();
}

template <int N, int V>
hipError_t col_variant(const Dims& d, int mode, const ColArgs& a, hipStream_t s) {
    switch (mode) {
        case COL_INIT: return col_mode<N, V, COL_INIT>(d, a, s);
        case COL_A: return col_mode<N, V, COL_A>(d, a, s);
        case COL_B: return col_mode<N, V, COL_B>(d, a, s);
        case COL_C: return col_mode<N, V, COL_C>(d, a, s);
        case COL_D: return col_mode<N, V, COL_D>(d, a, s);
        case COL_FILTER: return col_mode<N, V, COL_FILTER>(d, a, s);
        case COL_FROM_STATE: return col_mode<N, V, COL_FROM_STATE>(d, a, s);
        case COL_ADJ_C: return col_mode<N, V, COL_ADJ_C>(d, a, s);
        case COL_ADJ_B: return col_mode<N, V, COL_ADJ_B>(d, a, s);
        case COL_ADJ_A: return col_mode<N, V, COL_ADJ_A>(d, a, s);
        case COL_ADJ_N: return col_mode<N, V, COL_ADJ_N>(d, a, s);
        case COL_ADJ_NSRC: return col_mode<N, V, COL_ADJ_NSRC>(d, a, s);
        case COL_ADJ_SRC: return col_mode<N, V, COL_ADJ_SRC>(d, a, s);
        case COL_FIRST_GUESS: return col_mode<N, V, COL_FIRST_GUESS>(d, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t Launch<N>::col(const Dims& d, int mode, const ColArgs& a, hipStream_t s) {
    if (d.cvar == 0) return col_variant<N, 0>(d, mode, a, s);
    if (d.cvar == 1) return col_variant<N, 1>(d, mode, a, s);
    return col_variant<N, 2>(d, mode, a, s);
}

template <int N>
int Launch<N>::threads(int var) {
    return var == 0 ? Plan<N, 0>::T : var == 1 ? Plan<N, 1>::T : Plan<N, 2>::T;
}

}  // namespace pa
