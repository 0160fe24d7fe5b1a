// fft.hpp -- FP64 complex FFT building blocks for gfx950 (CDNA4).
//
// A length-N transform is done by a "team" of T threads.  Thread t of a team
// holds E = N / T elements in registers, element t + T*m in slot m (m < E).
// The transform is a Stockham autosort sequence of radix-R stages (R in
// {2, 4, 8, 16}); each stage does E/R butterflies per thread entirely in
// registers and, between stages, the team exchanges data through its own LDS
// region (one write + barrier + read per stage boundary).  The first stage's
// inputs and the last stage's outputs are both in the register layout
// "thread t holds index t + T*m", so a forward transform, a pointwise
// operation and an inverse transform chain with no extra exchange, and global
// loads/stores of a contiguous signal are coalesced across the team.
//
// Direction: forward uses exp(-2 pi i jk/N) (unnormalised), inverse
// exp(+2 pi i jk/N) (unnormalised).  Inter-stage twiddles come from a
// stage-ordered table in LDS (see twiddle_source) filled from the natural
// table exp(-2 pi i m / N), m < N, precomputed on the host.
#pragma once
#include <hip/hip_runtime.h>

namespace pa {

// 16-byte aligned so that LDS and global accesses of one value are single
// 128-bit operations (ds_read_b128: a lane covers four consecutive banks).
struct alignas(16) cd { double x, y; };

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS
// operations, then meets the other waves.  Unlike __syncthreads() it does not
// drain outstanding global loads, so loads issued before a transform stay in
// flight across its exchanges.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Hand-off inside one wavefront: a wave's LDS operations are executed in
// issue order, so a team that lies within one wave only has to wait for its
// own LDS operations (and keep the compiler from moving accesses across).
// No other wave is stalled.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// WL: the team lies within one wavefront (T divides 64 and teams are
// consecutive threads), so its exchanges need no workgroup barrier.
template <bool WL>
__device__ __forceinline__ void team_sync() {
    if constexpr (WL) wave_lds_sync();
    else lds_sync();
}

__device__ __forceinline__ cd mk(double x, double y) { cd r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd csub(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd cmul(cd a, cd b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cd cmulc(cd a, cd b) { return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }  // a*conj(b)
__device__ __forceinline__ cd cconj(cd a) { return mk(a.x, -a.y); }
__device__ __forceinline__ cd cscale(cd a, double s) { return mk(a.x * s, a.y * s); }
__device__ __forceinline__ cd mul_i(cd a) { return mk(-a.y, a.x); }     //  i a
__device__ __forceinline__ cd mul_mi(cd a) { return mk(a.y, -a.x); }    // -i a
__device__ __forceinline__ cd czero() { return mk(0.0, 0.0); }

// cos / sin of 2 pi k / 16, k = 0..15 (correctly rounded literals).
#define PA_C1 0.92387953251128675613
#define PA_S1 0.38268343236508977173
#define PA_R2 0.70710678118654752440

template <int K16>
struct Unit16 {
    static constexpr double c = (K16 % 16 == 0) ? 1.0 : (K16 % 16 == 1) ? PA_C1 : (K16 % 16 == 2) ? PA_R2
        : (K16 % 16 == 3) ? PA_S1 : (K16 % 16 == 4) ? 0.0 : (K16 % 16 == 5) ? -PA_S1 : (K16 % 16 == 6) ? -PA_R2
        : (K16 % 16 == 7) ? -PA_C1 : (K16 % 16 == 8) ? -1.0 : (K16 % 16 == 9) ? -PA_C1 : (K16 % 16 == 10) ? -PA_R2
        : (K16 % 16 == 11) ? -PA_S1 : (K16 % 16 == 12) ? 0.0 : (K16 % 16 == 13) ? PA_S1 : (K16 % 16 == 14) ? PA_R2
        : PA_C1;
    static constexpr double s = (K16 % 16 == 0) ? 0.0 : (K16 % 16 == 1) ? PA_S1 : (K16 % 16 == 2) ? PA_R2
        : (K16 % 16 == 3) ? PA_C1 : (K16 % 16 == 4) ? 1.0 : (K16 % 16 == 5) ? PA_C1 : (K16 % 16 == 6) ? PA_R2
        : (K16 % 16 == 7) ? PA_S1 : (K16 % 16 == 8) ? 0.0 : (K16 % 16 == 9) ? -PA_S1 : (K16 % 16 == 10) ? -PA_R2
        : (K16 % 16 == 11) ? -PA_C1 : (K16 % 16 == 12) ? -1.0 : (K16 % 16 == 13) ? -PA_C1 : (K16 % 16 == 14) ? -PA_R2
        : -PA_S1;
};

// a * exp(-+ 2 pi i K / R) with R dividing 16; exact special cases.
template <int K, int R, bool INV>
__device__ __forceinline__ cd twc(cd a) {
    constexpr int k16 = ((K * (16 / R)) % 16 + 16) % 16;
    if constexpr (k16 == 0) return a;
    else if constexpr (k16 == 8) return mk(-a.x, -a.y);
    else if constexpr (k16 == 4) return INV ? mul_i(a) : mul_mi(a);
    else if constexpr (k16 == 12) return INV ? mul_mi(a) : mul_i(a);
    else {
        constexpr double c = Unit16<k16>::c;
        constexpr double s = INV ? Unit16<k16>::s : -Unit16<k16>::s;
        return mk(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

template <bool INV>
__device__ __forceinline__ void dft2(cd& a, cd& b) {
    cd t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(cd& x0, cd& x1, cd& x2, cd& x3) {
    cd a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = csub(x1, x3);
    cd dd = INV ? mul_i(d) : mul_mi(d);
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, dd);
    x3 = csub(b, dd);
}

// In-place R-point DFT of v[0..R-1] with natural-order output.
template <int R, bool INV>
__device__ __forceinline__ void dft(cd* v);

template <>
__device__ __forceinline__ void dft<2, false>(cd* v) { dft2<false>(v[0], v[1]); }
template <>
__device__ __forceinline__ void dft<2, true>(cd* v) { dft2<true>(v[0], v[1]); }
template <>
__device__ __forceinline__ void dft<4, false>(cd* v) { dft4<false>(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void dft<4, true>(cd* v) { dft4<true>(v[0], v[1], v[2], v[3]); }

// 8 = 2 x 4:  X[k1 + 4 k2] = sum_p w8^{p k1} w2^{p k2} sum_m x[2m+p] w4^{m k1}
template <bool INV>
__device__ __forceinline__ void dft8(cd* v) {
    dft4<INV>(v[0], v[2], v[4], v[6]);
    dft4<INV>(v[1], v[3], v[5], v[7]);
    v[3] = twc<1, 8, INV>(v[3]);
    v[5] = twc<2, 8, INV>(v[5]);
    v[7] = twc<3, 8, INV>(v[7]);
    dft2<INV>(v[0], v[1]);
    dft2<INV>(v[2], v[3]);
    dft2<INV>(v[4], v[5]);
    dft2<INV>(v[6], v[7]);
    // v[2 k1 + k2] holds X[k1 + 4 k2]
    cd o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 2; ++k2) o[k1 + 4 * k2] = v[2 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = o[i];
}
template <>
__device__ __forceinline__ void dft<8, false>(cd* v) { dft8<false>(v); }
template <>
__device__ __forceinline__ void dft<8, true>(cd* v) { dft8<true>(v); }

// 16 = 4 x 4:  X[k1 + 4 k2] = sum_p w16^{p k1} w4^{p k2} sum_m x[4m+p] w4^{m k1}
template <bool INV>
__device__ __forceinline__ void dft16(cd* v) {
#pragma unroll
    for (int p = 0; p < 4; ++p) dft4<INV>(v[p], v[4 + p], v[8 + p], v[12 + p]);
    // v[p + 4 k1] = Y_p[k1]; twiddle by w16^{p k1}
    v[5] = twc<1, 16, INV>(v[5]);
    v[6] = twc<2, 16, INV>(v[6]);
    v[7] = twc<3, 16, INV>(v[7]);
    v[9] = twc<2, 16, INV>(v[9]);
    v[10] = twc<4, 16, INV>(v[10]);
    v[11] = twc<6, 16, INV>(v[11]);
    v[13] = twc<3, 16, INV>(v[13]);
    v[14] = twc<6, 16, INV>(v[14]);
    v[15] = twc<9, 16, INV>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]
    cd o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = o[i];
}
template <>
__device__ __forceinline__ void dft<16, false>(cd* v) { dft16<false>(v); }
template <>
__device__ __forceinline__ void dft<16, true>(cd* v) { dft16<true>(v); }

// ---------------------------------------------------------------- plans --
// Radix sequence per length and variant; T threads per transform, E elements
// per thread (every radix divides E).  Variant 0 keeps more elements per
// thread (fewer LDS exchanges, more registers); variant 1 spreads a transform
// over more threads; variant 2 uses four elements per thread where the
// length allows it (twice the threads of variant 1 at 128 and 256, the same
// plan as variant 1 elsewhere).  The autotuner picks per context and pass.
template <int N, int V> struct Plan;
template <int V> struct Plan<8, V>    { static constexpr int NS = 1, T = 1,  E = 8;  static constexpr int R[4] = {8, 1, 1, 1}; };
template <int V> struct Plan<16, V>   { static constexpr int NS = 2, T = 4,  E = 4;  static constexpr int R[4] = {4, 4, 1, 1}; };
template <int V> struct Plan<32, V>   { static constexpr int NS = 2, T = 4,  E = 8;  static constexpr int R[4] = {8, 4, 1, 1}; };
template <> struct Plan<64, 0>   { static constexpr int NS = 2, T = 8,   E = 8;  static constexpr int R[4] = {8, 8, 1, 1}; };
template <> struct Plan<64, 1>   { static constexpr int NS = 3, T = 16,  E = 4;  static constexpr int R[4] = {4, 4, 4, 1}; };
template <> struct Plan<64, 2>   { static constexpr int NS = 3, T = 16,  E = 4;  static constexpr int R[4] = {4, 4, 4, 1}; };
template <> struct Plan<128, 0>  { static constexpr int NS = 2, T = 8,   E = 16; static constexpr int R[4] = {16, 8, 1, 1}; };
template <> struct Plan<128, 1>  { static constexpr int NS = 3, T = 16,  E = 8;  static constexpr int R[4] = {8, 4, 4, 1}; };
template <> struct Plan<128, 2>  { static constexpr int NS = 4, T = 32,  E = 4;  static constexpr int R[4] = {4, 4, 4, 2}; };
template <> struct Plan<256, 0>  { static constexpr int NS = 2, T = 16,  E = 16; static constexpr int R[4] = {16, 16, 1, 1}; };
template <> struct Plan<256, 1>  { static constexpr int NS = 3, T = 32,  E = 8;  static constexpr int R[4] = {8, 8, 4, 1}; };
template <> struct Plan<256, 2>  { static constexpr int NS = 4, T = 64,  E = 4;  static constexpr int R[4] = {4, 4, 4, 4}; };
template <int V> struct Plan<512, V>  { static constexpr int NS = 3, T = 64, E = 8; static constexpr int R[4] = {8, 8, 8, 1}; };
template <> struct Plan<1024, 0> { static constexpr int NS = 3, T = 64,  E = 16; static constexpr int R[4] = {16, 16, 4, 1}; };
template <> struct Plan<1024, 1> { static constexpr int NS = 4, T = 128, E = 8;  static constexpr int R[4] = {8, 8, 4, 4}; };
template <> struct Plan<1024, 2> { static constexpr int NS = 4, T = 128, E = 8;  static constexpr int R[4] = {8, 8, 4, 4}; };

// LDS footprint of one team's exchange area (one padding slot per 16 entries).
template <int N>
__host__ __device__ constexpr int lds_team() { return N + N / 16 + 1; }
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Where entry i of a team's exchange lives.  A 16-byte LDS access is served
// a few lanes at a time, and lanes whose entries fall on the same bank group
// wait for each other.  The Stockham stages write with strides S R and read
// with stride 1, so no single layout serves all of them.  A plan may instead
// XOR the low four bits of i with i >> A ^ i >> B ^ i >> C (a bijection within
// each aligned block of 16 entries).  Counting bank groups over every exchange
// of a plan suggests such swizzles for most plans, but measured on gfx950 only
// the plans made of radix-4 stages gain (256 points: adjoint rows 46.3 -> 43.9
// us for 64 members; 128 points: 3-4 %); every plan with a radix-8 stage
// loses 8-26 % (128, 256, 512 and 1024 points) and 64 points is flat.  Those
// keep one padding slot per 16 entries.
template <int N, int V> struct LdsSwizzle { static constexpr int A = 0, B = 0, C = 0; };
template <> struct LdsSwizzle<128, 2>  { static constexpr int A = 2, B = 0, C = 0; };
template <> struct LdsSwizzle<256, 2>  { static constexpr int A = 2, B = 7, C = 0; };

template <int N, int V>
__device__ __forceinline__ int lpos(int i) {
    using Z = LdsSwizzle<N, V>;
    if constexpr (Z::A == 0) {
        return lpad(i);
    } else {
        int h = i >> Z::A;
        if constexpr (Z::B != 0) h ^= i >> Z::B;
        if constexpr (Z::C != 0) h ^= i >> Z::C;
        return (i & ~15) | ((i ^ h) & 15);
    }
}

// Stage-ordered twiddle table.  The factor exp(-2 pi i r k / (S R)) of the
// stage with span S and radix R (1 <= r < R, 0 <= k < S) sits at r S + k - 1;
// the stages' ranges [S - 1, S R - 1) tile [0, N - 1).  Lanes of a stage hold
// consecutive k, so they read consecutive entries (no bank conflicts), where
// the natural table indexed by r k N / (S R) puts them on a few banks.
// Returns the natural-table index of stage-ordered entry n.
template <int N, int V>
__host__ __device__ constexpr int twiddle_source(int n) {
    using P = Plan<N, V>;
    int S = 1;
    for (int s = 0; s < P::NS; ++s) {
        const int R = P::R[s];
        if (n + 1 < S * R) return ((n + 1) / S) * ((n + 1) % S) * (N / (S * R));
        S *= R;
    }
    return 0;
}

// One Stockham stage: radix R, span S (product of the radices already done).
template <int N, int V, int R, int S, bool INV, bool LAST, bool WL>
__device__ __forceinline__ void fft_stage(cd* v, int t, cd* lds, const cd* __restrict__ tw) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + T * b;
        cd u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[b + r * NB];
        if constexpr (S > 1) {
            const int k = j % S;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cd w = tw[r * S + k - 1];
                u[r] = INV ? cmulc(u[r], w) : cmul(u[r], w);
            }
        }
        dft<R, INV>(u);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + r * NB] = u[r];
        } else {
            const int base = (j / S) * S * R + (j % S);
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lpos<N, V>(base + r * S)] = u[r];
        }
    }
    if constexpr (!LAST) {
        team_sync<WL>();
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = lds[lpos<N, V>(t + T * m)];
        team_sync<WL>();
    }
}

// Full transform of the team's register signal v (layout t + T*m).
// Unless WL, every thread of the workgroup must call this (it contains
// barriers when the plan has more than one stage).
template <int N, int V, bool INV, bool WL = false>
__device__ __forceinline__ void fft(cd* v, int t, cd* lds, const cd* __restrict__ tw) {
    using P = Plan<N, V>;
    constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
    if constexpr (P::NS == 1) {
        fft_stage<N, V, R0, 1, INV, true, WL>(v, t, lds, tw);
    } else if constexpr (P::NS == 2) {
        fft_stage<N, V, R0, 1, INV, false, WL>(v, t, lds, tw);
        fft_stage<N, V, R1, R0, INV, true, WL>(v, t, lds, tw);
    } else if constexpr (P::NS == 3) {
        fft_stage<N, V, R0, 1, INV, false, WL>(v, t, lds, tw);
        fft_stage<N, V, R1, R0, INV, false, WL>(v, t, lds, tw);
        fft_stage<N, V, R2, R0 * R1, INV, true, WL>(v, t, lds, tw);
    } else {
        fft_stage<N, V, R0, 1, INV, false, WL>(v, t, lds, tw);
        fft_stage<N, V, R1, R0, INV, false, WL>(v, t, lds, tw);
        fft_stage<N, V, R2, R0 * R1, INV, false, WL>(v, t, lds, tw);
        fft_stage<N, V, R3, R0 * R1 * R2, INV, true, WL>(v, t, lds, tw);
    }
}

// ---- transforms with the thread's twiddles held in registers ----
// A kernel that runs several transforms of one plan per row reads each
// twiddle factor from LDS once: the factors a thread needs depend only on the
// plan and its index t, not on the data, and the compiler reloads an LDS
// table after every exchange because the exchange stores may alias it.
// Stage q (q >= 1, span S = R[0] ... R[q-1]) keeps NB (R[q] - 1) factors at
// offset tw_reg_offset(q); all indices are compile-time, so the array stays
// in registers.  Results are bitwise those of fft().
template <int N, int V>
constexpr int tw_reg_offset(int q) {
    int o = 0;
    for (int s = 1; s < q; ++s) o += (Plan<N, V>::E / Plan<N, V>::R[s]) * (Plan<N, V>::R[s] - 1);
    return o;
}
template <int N, int V>
struct TwReg {
    static constexpr int COUNT = tw_reg_offset<N, V>(Plan<N, V>::NS);
    cd w[COUNT > 0 ? COUNT : 1];
};

template <int N, int V, int Q, int S>
__device__ __forceinline__ void load_tw_stage(cd* w, int t, const cd* __restrict__ tw) {
    constexpr int T = Plan<N, V>::T, R = Plan<N, V>::R[Q], NB = Plan<N, V>::E / R;
    constexpr int OFF = tw_reg_offset<N, V>(Q);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int k = (t + T * b) % S;
#pragma unroll
        for (int r = 1; r < R; ++r) w[OFF + b * (R - 1) + r - 1] = tw[r * S + k - 1];
    }
}

template <int N, int V>
__device__ __forceinline__ void load_twiddles(TwReg<N, V>& tr, int t, const cd* __restrict__ tw) {
    using P = Plan<N, V>;
    constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2];
    if constexpr (P::NS >= 2) load_tw_stage<N, V, 1, R0>(tr.w, t, tw);
    if constexpr (P::NS >= 3) load_tw_stage<N, V, 2, R0 * R1>(tr.w, t, tw);
    if constexpr (P::NS >= 4) load_tw_stage<N, V, 3, R0 * R1 * R2>(tr.w, t, tw);
}

template <int N, int V, int R, int S, int OFF, bool INV, bool LAST, bool WL>
__device__ __forceinline__ void fft_stage_reg(cd* v, int t, cd* lds, const cd* w) {
    constexpr int T = Plan<N, V>::T, E = Plan<N, V>::E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + T * b;
        cd u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[b + r * NB];
        if constexpr (S > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cd f = w[OFF + b * (R - 1) + r - 1];
                u[r] = INV ? cmulc(u[r], f) : cmul(u[r], f);
            }
        }
        dft<R, INV>(u);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + r * NB] = u[r];
        } else {
            const int base = (j / S) * S * R + (j % S);
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lpos<N, V>(base + r * S)] = u[r];
        }
    }
    if constexpr (!LAST) {
        team_sync<WL>();
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = lds[lpos<N, V>(t + T * m)];
        team_sync<WL>();
    }
}

template <int N, int V, bool INV, bool WL = false>
__device__ __forceinline__ void fft(cd* v, int t, cd* lds, const TwReg<N, V>& tr) {
    using P = Plan<N, V>;
    constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
    constexpr int O1 = tw_reg_offset<N, V>(1), O2 = tw_reg_offset<N, V>(2), O3 = tw_reg_offset<N, V>(3);
    if constexpr (P::NS == 1) {
        fft_stage_reg<N, V, R0, 1, 0, INV, true, WL>(v, t, lds, tr.w);
    } else if constexpr (P::NS == 2) {
        fft_stage_reg<N, V, R0, 1, 0, INV, false, WL>(v, t, lds, tr.w);
        fft_stage_reg<N, V, R1, R0, O1, INV, true, WL>(v, t, lds, tr.w);
    } else if constexpr (P::NS == 3) {
        fft_stage_reg<N, V, R0, 1, 0, INV, false, WL>(v, t, lds, tr.w);
        fft_stage_reg<N, V, R1, R0, O1, INV, false, WL>(v, t, lds, tr.w);
        fft_stage_reg<N, V, R2, R0 * R1, O2, INV, true, WL>(v, t, lds, tr.w);
    } else {
        fft_stage_reg<N, V, R0, 1, 0, INV, false, WL>(v, t, lds, tr.w);
        fft_stage_reg<N, V, R1, R0, O1, INV, false, WL>(v, t, lds, tr.w);
        fft_stage_reg<N, V, R2, R0 * R1, O2, INV, false, WL>(v, t, lds, tr.w);
        fft_stage_reg<N, V, R3, R0 * R1 * R2, O3, INV, true, WL>(v, t, lds, tr.w);
    }
}

// ---- 256 points on one wavefront with cross-lane digit exchanges (gfx950) ----
// A row of 256 points is held by the 64 lanes of one wavefront, four values per
// lane: element t + 64 m in register m of lane t (the layout of plan (256, 2)).
// Writing an index in base 4 as i = i0 + 4 i1 + 16 i2 + 64 i3, lane t holds the
// digits (i0, i1, i2) and register m the digit i3.  The transform runs four
// radix-4 decimation-in-frequency stages; each needs the digit it transforms in
// the register, so between stages the register digit trades places with one
// lane digit:
//   * i2 (lane bits 5:4) through the gfx950 lane-swap instructions, which run
//     on the vector ALU and need no LDS: v_permlane32_swap trades lane bit 5
//     with register bit 1, v_permlane16_swap lane bit 4 with register bit 0;
//   * i1 and then i0 through LDS, in layouts where the 16 lanes of any aligned
//     group write and read 16 distinct 16-byte slots (a XOR of the slot's low
//     bits with the register index), so no access waits on a bank;
// and the last exchange also places the output in natural order (element k in
// register k / 64 of lane k mod 64).  Input and output therefore share the
// layout of the Stockham plan, and chain with the pointwise products in the
// same way, with one LDS exchange fewer per transform.
// Twiddles (DIF): after the stage on digit i3 the output of digit k0 is
// multiplied by w256^(k0 n1) (n1 = i0 + 4 i1 + 16 i2), after the stage on i2
// by w64^(k1 n2) (n2 = i0 + 4 i1), after the stage on i1 by w16^(k2 i0).
struct Tw256 {
    cd w[9];
};

// The thread's nine factors from the natural table tw[m] = exp(-2 pi i m / 256).
__device__ __forceinline__ void load_tw256(Tw256& tr, int t, const cd* __restrict__ tw) {
    const int n2 = t & 15, i0 = t & 3;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        tr.w[k - 1] = tw[(k * t) & 255];
        tr.w[2 + k] = tw[(4 * k * n2) & 255];
        tr.w[5 + k] = tw[(16 * k * i0) & 255];
    }
}

// Lanes 32-63 of a trade places with lanes 0-31 of b (one v_permlane32_swap per dword).
__device__ __forceinline__ void lane_swap32(double& a, double& b) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | (unsigned long long)lo[0]);
    b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | (unsigned long long)lo[1]);
}
// The odd 16-lane rows of a trade places with the even rows of b (v_permlane16_swap).
__device__ __forceinline__ void lane_swap16(double& a, double& b) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | (unsigned long long)lo[0]);
    b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | (unsigned long long)lo[1]);
}

template <bool INV>
__device__ __forceinline__ cd tw_apply(cd a, cd w) { return INV ? cmulc(a, w) : cmul(a, w); }

// The transform of the wavefront's row (v: the lane's 4 values; lds: the
// wavefront's 256-entry exchange area).  Every lane of the wavefront must be
// active.  Forward: exp(-2 pi i jk / 256); INV: exp(+2 pi i jk / 256).
template <bool INV>
__device__ __forceinline__ void fft256_wave(cd* v, int t, cd* lds, const Tw256& tr) {
    // stage on i3 (in the register)
    dft4<INV>(v[0], v[1], v[2], v[3]);
    v[1] = tw_apply<INV>(v[1], tr.w[0]);
    v[2] = tw_apply<INV>(v[2], tr.w[1]);
    v[3] = tw_apply<INV>(v[3], tr.w[2]);
    // register digit k0 <-> lane digit i2 (bits 5:4): (reg, lane) = (i2, n2 + 16 k0)
    lane_swap32(v[0].x, v[2].x);
    lane_swap32(v[0].y, v[2].y);
    lane_swap32(v[1].x, v[3].x);
    lane_swap32(v[1].y, v[3].y);
    lane_swap16(v[0].x, v[1].x);
    lane_swap16(v[0].y, v[1].y);
    lane_swap16(v[2].x, v[3].x);
    lane_swap16(v[2].y, v[3].y);
    // stage on i2
    dft4<INV>(v[0], v[1], v[2], v[3]);
    v[1] = tw_apply<INV>(v[1], tr.w[3]);
    v[2] = tw_apply<INV>(v[2], tr.w[4]);
    v[3] = tw_apply<INV>(v[3], tr.w[5]);
    // (reg, lane) = (k1, i0 + 4 i1 + 16 k0) -> (i1, i0 + 4 k1 + 16 k0); slot 64 reg + (lane ^ 4 reg)
    {
        const int i1 = (t >> 2) & 3, keep = t & 0x33;
#pragma unroll
        for (int r = 0; r < 4; ++r) lds[64 * i1 + ((keep | (r << 2)) ^ (i1 << 2))] = v[r];
        wave_lds_sync();
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] = lds[64 * m + (t ^ (m << 2))];
        wave_lds_sync();
    }
    // stage on i1
    dft4<INV>(v[0], v[1], v[2], v[3]);
    v[1] = tw_apply<INV>(v[1], tr.w[6]);
    v[2] = tw_apply<INV>(v[2], tr.w[7]);
    v[3] = tw_apply<INV>(v[3], tr.w[8]);
    // (reg, lane) = (k2, i0 + 4 k1 + 16 k0) -> (i0, k0 + 4 k1 + 16 k2); slot 64 reg + (lane ^ reg)
    {
        const int i0 = t & 3, kk = (t >> 4) | (t & 12);
#pragma unroll
        for (int r = 0; r < 4; ++r) lds[64 * i0 + ((kk | (r << 4)) ^ i0)] = v[r];
        wave_lds_sync();
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] = lds[64 * m + (t ^ m)];
        wave_lds_sync();
    }
    // stage on i0: register m now holds X[t + 64 m]
    dft4<INV>(v[0], v[1], v[2], v[3]);
}

}  // namespace pa
