// kernels.hip -- row (physical-space) and column (spectral-space) passes.
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
#include "kernels.hpp"

namespace pa {

// z = A_full[e] + i B_full[e] for the Hermitian extensions of half-spectrum
// rows A, B (only kx = 0..K stored, zero beyond).  The kx = 0 entry of a real
// field's half spectrum is real; its imaginary round-off is discarded.
__device__ __forceinline__ cd herm_pair(const cd* __restrict__ A, const cd* __restrict__ B, int e,
                                        int N, int K) {
    if (e == 0) return mk(A[0].x, B[0].x);
    if (e <= K) {
        const cd a = A[e], b = B[e];
        return mk(a.x - b.y, a.y + b.x);
    }
    if (e >= N - K) {
        const cd a = A[N - e], b = B[N - e];
        return mk(a.x + b.y, b.x - a.y);
    }
    return czero();
}

__device__ __forceinline__ cd herm_single(const cd* __restrict__ A, int e, int N, int K) {
    if (e == 0) return mk(A[0].x, 0.0);
    if (e <= K) return A[e];
    if (e >= N - K) return cconj(A[N - e]);
    return czero();
}

// Forward transform z of a + i b (a, b real) is split into the half spectra
// of a and b:  Ahat[k] = (Z[k] + conj Z[N-k]) / 2,  Bhat[k] = (Z[k] - conj Z[N-k]) / (2i).
// Stores kx = 0..K of both.  Called by every thread of the workgroup.
template <int N>
__device__ __forceinline__ void split_store(const cd* z, int t, cd* lds, cd* __restrict__ outA,
                                            cd* __restrict__ outB, int K) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
#pragma unroll
    for (int m = 0; m < E; ++m) lds[lpad(t + T * m)] = z[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + T * m;
        if (k <= K) {
            const cd zk = z[m];
            const cd zn = lds[lpad((N - k) & (N - 1))];
            outA[k] = mk(0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y));
            outB[k] = mk(0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x));
        }
    }
    __syncthreads();
}

// Team sum (fixed order) of one double per thread; result valid in thread t == 0.
template <int N>
__device__ __forceinline__ double team_sum(double v, int t, cd* lds) {
    constexpr int T = Plan<N>::T;
    lds[t] = mk(v, 0.0);
    __syncthreads();
    double s = 0.0;
    if (t == 0)
        for (int i = 0; i < T; ++i) s += lds[i].x;
    __syncthreads();
    return s;
}

// ------------------------------------------------------------ row passes --

// physical rows (y0, y0+1) -> Y rows; team per row pair.
template <int N>
__global__ void __launch_bounds__(256) row_r2c_kernel(Dims d, const double* __restrict__ in,
                                                      cd* __restrict__ out, const cd* __restrict__ tw) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int team = threadIdx.x / T, t = threadIdx.x % T;
    cd* lds = smem + team * lds_team<N>();
    const int g = blockIdx.x * (blockDim.x / T) + team;
    const int b = g / (N / 2), y0 = 2 * (g % (N / 2));
    const double* r0 = in + ((size_t)b * N + y0) * N;
    cd z[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + T * m;
        z[m] = mk(r0[x], r0[N + x]);
    }
    fft<N, false>(z, t, lds, tw);
    cd* o0 = out + ((size_t)b * N + y0) * d.KXP;
    split_store<N>(z, t, lds, o0, o0 + d.KXP, d.K);
}

// Y rows (y0, y0+1) -> physical rows.
template <int N>
__global__ void __launch_bounds__(256) row_c2r_kernel(Dims d, const cd* __restrict__ in,
                                                      double* __restrict__ out, const cd* __restrict__ tw) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int team = threadIdx.x / T, t = threadIdx.x % T;
    cd* lds = smem + team * lds_team<N>();
    const int g = blockIdx.x * (blockDim.x / T) + team;
    const int b = g / (N / 2), y0 = 2 * (g % (N / 2));
    const cd* i0 = in + ((size_t)b * N + y0) * d.KXP;
    cd z[E];
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = herm_pair(i0, i0 + d.KXP, t + T * m, N, d.K);
    fft<N, true>(z, t, lds, tw);
    double* r0 = out + ((size_t)b * N + y0) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + T * m;
        r0[x] = z[m].x;
        r0[N + x] = z[m].y;
    }
}

// Observation of (u, v) on one row: residual against the values, model
// observations out, and this thread's share of sum |r|^2.
__device__ __forceinline__ double observe_row(const RowObs& o, int b, int y, int x, double u, double v) {
    if ((y % o.stride) != 0 || (x % o.stride) != 0) return 0.0;
    const int i = x / o.stride, j = y / o.stride, M = o.M;
    const size_t base = (((size_t)b * o.n_times + o.slot) * 2) * M * M + (size_t)j * M + i;
    if (o.obs_out) {
        o.obs_out[base] = u;
        o.obs_out[base + (size_t)M * M] = v;
    }
    if (!o.values) return 0.0;
    const double ru = u - o.values[base];
    const double rv = v - o.values[base + (size_t)M * M];
    return ru * ru + rv * rv;
}

__device__ __forceinline__ void store_jpart(const RowObs& o, int b, int y, double s) {
    if (o.jpart && o.values && (y % o.stride) == 0)
        o.jpart[((size_t)b * o.n_times + o.slot) * o.M + y / o.stride] = 0.5 * s;
}

// Right-hand side products of one row:  q = u w_x + v w_y  (+ observation).
// Inputs yin[0..3] = U, V, Wx, Wy (Y layout), output yout[0] = row transform of q.
template <int N>
__global__ void __launch_bounds__(256) row_nl_kernel(Dims d, RowArgs a) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int team = threadIdx.x / T, t = threadIdx.x % T;
    cd* lds = smem + team * lds_team<N>();
    const int g = blockIdx.x * (blockDim.x / T) + team;
    const int b = g / N, y = g % N;
    const size_t roff = ((size_t)b * N + y) * d.KXP;
    cd z1[E], z2[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + T * m;
        z1[m] = herm_pair(a.yin[0] + roff, a.yin[2] + roff, e, N, d.K);   // u + i w_x
        z2[m] = herm_pair(a.yin[1] + roff, a.yin[3] + roff, e, N, d.K);   // v + i w_y
    }
    fft<N, true>(z1, t, lds, a.tw);
    fft<N, true>(z2, t, lds, a.tw);
    double part = 0.0;
    const bool obs = a.obs.slot >= 0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const double u = z1[m].x, wx = z1[m].y, v = z2[m].x, wy = z2[m].y;
        if (obs) part += observe_row(a.obs, b, y, t + T * m, u, v);
        z1[m] = mk(u * wx + v * wy, 0.0);
    }
    if (obs) {
        const double s = team_sum<N>(part, t, lds);
        if (t == 0) store_jpart(a.obs, b, y, s);
    }
    fft<N, false>(z1, t, lds, a.tw);
    cd* o = a.yout[0] + roff;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + T * m;
        if (k <= d.K) o[k] = z1[m];
    }
}

// Observation only (final time): team per observed row; yin[0..1] = U, V.
template <int N>
__global__ void __launch_bounds__(256) row_obs_kernel(Dims d, RowArgs a) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int team = threadIdx.x / T, t = threadIdx.x % T;
    cd* lds = smem + team * lds_team<N>();
    const int g = blockIdx.x * (blockDim.x / T) + team;
    const int b = g / a.obs.M, y = (g % a.obs.M) * a.obs.stride;
    const size_t roff = ((size_t)b * N + y) * d.KXP;
    cd z[E];
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = herm_pair(a.yin[0] + roff, a.yin[1] + roff, t + T * m, N, d.K);
    fft<N, true>(z, t, lds, a.tw);
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) part += observe_row(a.obs, b, y, t + T * m, z[m].x, z[m].y);
    const double s = team_sum<N>(part, t, lds);
    if (t == 0) store_jpart(a.obs, b, y, s);
}

// Adjoint products of one row.  yin[0..3] = U, V, Wx, Wy of the stage state,
// yin[4] = Lambda (the projected cotangent).  Outputs (row transforms):
//   yout[0] = w_x Lam - S^T r_u,  yout[1] = w_y Lam - S^T r_v,
//   yout[2] = u Lam,              yout[3] = v Lam
// with the observation residual r only when obs.slot >= 0 (stage n of an
// observed step): the source U^T S^T r_u + V^T S^T r_v rides on the first two
// products because it meets the same transposed multipliers.
template <int N>
__global__ void __launch_bounds__(256) row_adj_kernel(Dims d, RowArgs a) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int team = threadIdx.x / T, t = threadIdx.x % T;
    cd* lds = smem + team * lds_team<N>();
    const int g = blockIdx.x * (blockDim.x / T) + team;
    const int b = g / N, y = g % N;
    const size_t roff = ((size_t)b * N + y) * d.KXP;
    double L[E];
    {
        cd z[E];
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = herm_single(a.yin[4] + roff, t + T * m, N, d.K);
        fft<N, true>(z, t, lds, a.tw);
#pragma unroll
        for (int m = 0; m < E; ++m) L[m] = z[m].x;
    }
    cd z1[E], z2[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + T * m;
        z1[m] = herm_pair(a.yin[0] + roff, a.yin[2] + roff, e, N, d.K);
        z2[m] = herm_pair(a.yin[1] + roff, a.yin[3] + roff, e, N, d.K);
    }
    fft<N, true>(z1, t, lds, a.tw);
    fft<N, true>(z2, t, lds, a.tw);
    const RowObs& o = a.obs;
    const bool src = o.slot >= 0 && o.values != nullptr && (y % o.stride) == 0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const double u = z1[m].x, wx = z1[m].y, v = z2[m].x, wy = z2[m].y;
        double A = wx * L[m], Bv = wy * L[m];
        const int x = t + T * m;
        if (src && (x % o.stride) == 0) {
            const int i = x / o.stride, j = y / o.stride, M = o.M;
            const size_t base = (((size_t)b * o.n_times + o.slot) * 2) * M * M + (size_t)j * M + i;
            A -= u - o.values[base];
            Bv -= v - o.values[base + (size_t)M * M];
        }
        z1[m] = mk(A, Bv);
        z2[m] = mk(u * L[m], v * L[m]);
    }
    fft<N, false>(z1, t, lds, a.tw);
    split_store<N>(z1, t, lds, a.yout[0] + roff, a.yout[1] + roff, d.K);
    fft<N, false>(z2, t, lds, a.tw);
    split_store<N>(z2, t, lds, a.yout[2] + roff, a.yout[3] + roff, d.K);
}

// Terminal adjoint source.  mode 0: observation residual at the final step
// (yin[0..1] = U, V of omega_H); mode 1: unit u-impulse at (imp_x, imp_y).
// Outputs yout[0] = -S^T r_u, yout[1] = -S^T r_v (row transforms).
template <int N>
__global__ void __launch_bounds__(256) row_src_kernel(Dims d, RowArgs a, int impulse) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int team = threadIdx.x / T, t = threadIdx.x % T;
    cd* lds = smem + team * lds_team<N>();
    const int g = blockIdx.x * (blockDim.x / T) + team;
    const int b = g / N, y = g % N;
    const size_t roff = ((size_t)b * N + y) * d.KXP;
    const RowObs& o = a.obs;
    cd z[E];
    if (!impulse) {
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = herm_pair(a.yin[0] + roff, a.yin[1] + roff, t + T * m, N, d.K);
        fft<N, true>(z, t, lds, a.tw);
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
            Bv = -(z[m].y - o.values[base + (size_t)M * M]);
        }
        z[m] = mk(A, Bv);
    }
    fft<N, false>(z, t, lds, a.tw);
    split_store<N>(z, t, lds, a.yout[0] + roff, a.yout[1] + roff, d.K);
}

// ---------------------------------------------------------- column pass --

__device__ __forceinline__ int band_row(int q, int N, int K, int KY) {
    if (q <= K) return q;
    if (q >= N - K) return q - N + KY;
    return -1;
}

template <int N, int MODE>
__global__ void __launch_bounds__(256) col_kernel(Dims d, ColArgs a) {
    constexpr int T = Plan<N>::T, E = Plan<N>::E;
    extern __shared__ cd smem[];
    const int CB = d.cb;
    const int c = threadIdx.x % CB, t = threadIdx.x / CB;
    cd* lds = smem + c * lds_team<N>();
    const int b = blockIdx.y;
    const int kx = blockIdx.x * CB + c;
    const int K = d.K, KXP = d.KXP, KY = d.KY;
    const bool colok = kx <= K;
    const size_t ybase = (size_t)b * N * KXP + kx;
    const size_t cbase = (size_t)b * KY * KXP + kx;
    const double dkx = (double)kx;
    const double ex = a.ex2[kx];
    const double h = a.h;

    int rr[E];
    bool ins[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int q = t + T * m;
        const int r = colok ? band_row(q, N, K, KY) : -1;
        rr[m] = r;
        ins[m] = r >= 0 && !(kx == 0 && r == 0);
    }

    cd w[E];   // spectral values handed to the output transforms

    if constexpr (MODE <= COL_FILTER) {
        cd v[E];
#pragma unroll
        for (int m = 0; m < E; ++m)
            v[m] = colok ? a.yin[0][ybase + (size_t)(t + T * m) * KXP] : czero();
        fft<N, false>(v, t, lds, a.tw);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rr[m];
            if (r < 0) { w[m] = czero(); continue; }
            const size_t ci = cbase + (size_t)r * KXP;
            if constexpr (MODE == COL_INIT) {
                const cd s = ins[m] ? v[m] : czero();
                a.omega[ci] = s;
                if (a.ckpt) a.ckpt[ci] = s;
                w[m] = s;
            } else if constexpr (MODE == COL_FILTER) {
                const size_t mi = (a.mult_per_member ? (size_t)b * KY * KXP : 0) + (size_t)r * KXP + kx;
                w[m] = ins[m] ? cscale(v[m], a.mult[mi]) : czero();
            } else {
                const int ky = (r <= K) ? r : r - KY;
                cd nl = ins[m] ? mk(-v[m].x, -v[m].y) : czero();
                if (a.nf > 0 && kx == 0 && (ky == a.nf || ky == -a.nf)) nl.x += a.forcing;
                const double e2 = ex * a.ey2[r];
                const double e1 = e2 * e2;
                const cd wn = a.omega[ci];
                if constexpr (MODE == COL_A) {
                    a.acc[ci] = cscale(nl, e1);
                    w[m] = cscale(mk(wn.x + 0.5 * h * nl.x, wn.y + 0.5 * h * nl.y), e2);
                } else if constexpr (MODE == COL_B) {
                    const cd ac = a.acc[ci];
                    a.acc[ci] = mk(ac.x + 2.0 * e2 * nl.x, ac.y + 2.0 * e2 * nl.y);
                    w[m] = mk(e2 * wn.x + 0.5 * h * nl.x, e2 * wn.y + 0.5 * h * nl.y);
                } else if constexpr (MODE == COL_C) {
                    const cd ac = a.acc[ci];
                    a.acc[ci] = mk(ac.x + 2.0 * e2 * nl.x, ac.y + 2.0 * e2 * nl.y);
                    w[m] = mk(e1 * wn.x + h * e2 * nl.x, e1 * wn.y + h * e2 * nl.y);
                } else {   // COL_D
                    const cd ac = a.acc[ci];
                    const double h6 = h / 6.0;
                    const cd s = mk(e1 * wn.x + h6 * (ac.x + nl.x), e1 * wn.y + h6 * (ac.y + nl.y));
                    a.omega[ci] = s;
                    if (a.ckpt) a.ckpt[ci] = s;
                    w[m] = s;
                }
            }
        }
    } else if constexpr (MODE == COL_FROM_STATE) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rr[m];
            if (r < 0) { w[m] = czero(); continue; }
            const size_t ci = cbase + (size_t)r * KXP;
            const cd s = ins[m] ? a.state_in[ci] : czero();
            if (a.omega) a.omega[ci] = s;
            w[m] = s;
        }
    } else {
        // adjoint: wbar = 1_S [ (i ky/k^2) A - (i kx/k^2) B + i kx C + i ky D ]
        constexpr int NIN = (MODE == COL_ADJ_SRC) ? 2 : 4;
        cd s[E];
#pragma unroll
        for (int m = 0; m < E; ++m) s[m] = czero();
#pragma unroll
        for (int p = 0; p < NIN; ++p) {
            cd v[E];
#pragma unroll
            for (int m = 0; m < E; ++m)
                v[m] = colok ? a.yin[p][ybase + (size_t)(t + T * m) * KXP] : czero();
            fft<N, false>(v, t, lds, a.tw);
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (!ins[m]) continue;
                const int r = rr[m];
                const double ky = (double)((r <= K) ? r : r - KY);
                const double ik2 = a.invk2[(size_t)r * KXP + kx];
                const double f = (p == 0) ? ky * ik2 : (p == 1) ? -dkx * ik2 : (p == 2) ? dkx : ky;
                s[m].x += f * v[m].x;
                s[m].y += f * v[m].y;
            }
        }
        const double sc = a.scale ? a.scale[b] : 1.0;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int r = rr[m];
            if (r < 0) { w[m] = czero(); continue; }
            const size_t ci = cbase + (size_t)r * KXP;
            const cd wb = ins[m] ? mul_i(s[m]) : czero();
            const double e2 = ex * a.ey2[r];
            const double e1 = e2 * e2;
            if constexpr (MODE == COL_ADJ_C) {
                const cd lm = a.lam[ci];
                a.omb[ci] = mk(e1 * (lm.x + wb.x), e1 * (lm.y + wb.y));
                w[m] = mk((h / 3.0) * e2 * lm.x + h * e2 * wb.x, (h / 3.0) * e2 * lm.y + h * e2 * wb.y);
            } else if constexpr (MODE == COL_ADJ_B) {
                const cd lm = a.lam[ci], ob = a.omb[ci];
                a.omb[ci] = mk(ob.x + e2 * wb.x, ob.y + e2 * wb.y);
                w[m] = mk((h / 3.0) * e2 * lm.x + 0.5 * h * wb.x, (h / 3.0) * e2 * lm.y + 0.5 * h * wb.y);
            } else if constexpr (MODE == COL_ADJ_A) {
                const cd lm = a.lam[ci], ob = a.omb[ci];
                a.omb[ci] = mk(ob.x + e2 * wb.x, ob.y + e2 * wb.y);
                w[m] = mk((h / 6.0) * e1 * lm.x + 0.5 * h * e2 * wb.x, (h / 6.0) * e1 * lm.y + 0.5 * h * e2 * wb.y);
            } else {   // COL_ADJ_N, COL_ADJ_SRC
                cd ln = wb;
                if constexpr (MODE == COL_ADJ_N) {
                    const cd ob = a.omb[ci];
                    ln = mk(ob.x + wb.x, ob.y + wb.y);
                }
                a.lam[ci] = ln;
                w[m] = a.final_out ? cscale(ln, sc) : cscale(ln, h / 6.0);
            }
        }
    }

    // derived fields: 1_S * multiplier * w / N^2, inverse transform along y
    const double inv_n2 = 1.0 / ((double)N * (double)N);
    for (int o = 0; o < a.nout; ++o) {
        const int f = a.fields[o];
        cd v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (!ins[m]) { v[m] = czero(); continue; }
            const int r = rr[m];
            const double ky = (double)((r <= K) ? r : r - KY);
            const cd s = cscale(w[m], inv_n2);
            if (f == F_OMEGA) v[m] = s;
            else if (f == F_U) v[m] = cscale(mul_i(s), ky * a.invk2[(size_t)r * KXP + kx]);
            else if (f == F_V) v[m] = cscale(mul_i(s), -dkx * a.invk2[(size_t)r * KXP + kx]);
            else if (f == F_WX) v[m] = cscale(mul_i(s), dkx);
            else v[m] = cscale(mul_i(s), ky);
        }
        fft<N, true>(v, t, lds, a.tw);
        if (colok) {
            cd* out = a.yout[o] + ybase;
#pragma unroll
            for (int m = 0; m < E; ++m) out[(size_t)(t + T * m) * KXP] = v[m];
        }
    }
}

// ------------------------------------------------------------- launchers --

// Host-side pointer checks: a launch whose buffers are missing is refused
// before it can touch memory.
static bool obs_ok(const RowObs& o) {
    if (o.slot < 0) return true;
    return o.stride >= 1 && o.M >= 1 && o.n_times > o.slot;
}

static bool col_ptrs_ok(int mode, const ColArgs& a) {
    if (!a.invk2 || !a.ex2 || !a.ey2 || !a.tw) return false;
    if (a.nout < 0 || a.nout > 4) return false;
    for (int o = 0; o < a.nout; ++o)
        if (!a.yout[o]) return false;
    switch (mode) {
        case COL_INIT: return a.yin[0] && a.omega;
        case COL_A: case COL_B: case COL_C: case COL_D: return a.yin[0] && a.omega && a.acc;
        case COL_FILTER: return a.yin[0] && a.mult;
        case COL_FROM_STATE: return a.state_in != nullptr;
        case COL_ADJ_C: case COL_ADJ_B: case COL_ADJ_A: case COL_ADJ_N:
            return a.yin[0] && a.yin[1] && a.yin[2] && a.yin[3] && a.lam && a.omb;
        case COL_ADJ_SRC: return a.yin[0] && a.yin[1] && a.lam;
        default: return false;
    }
}

template <int N>
static int row_teams(const Dims& d, long teams) {
    int tpb = d.tpb;
    const int cap = 256 / Plan<N>::T;
    if (tpb > cap) tpb = cap;
    if (tpb < 1) tpb = 1;
    while (tpb > 1 && (size_t)tpb * lds_team<N>() * sizeof(cd) > 65536) tpb >>= 1;
    while (tpb > 1 && teams % tpb) tpb >>= 1;
    return tpb;
}

template <int N>
static size_t row_lds(int tpb) { return (size_t)tpb * lds_team<N>() * sizeof(cd); }

#define PA_DISPATCH_N(N_, CALL)                      \
    switch (N_) {                                    \
        case 8: { constexpr int NN = 8; CALL; } break;       \
        case 16: { constexpr int NN = 16; CALL; } break;     \
        case 32: { constexpr int NN = 32; CALL; } break;     \
        case 64: { constexpr int NN = 64; CALL; } break;     \
        case 128: { constexpr int NN = 128; CALL; } break;   \
        case 256: { constexpr int NN = 256; CALL; } break;   \
        case 512: { constexpr int NN = 512; CALL; } break;   \
        case 1024: { constexpr int NN = 1024; CALL; } break; \
        default: return hipErrorInvalidValue;        \
    }

template <int N>
static hipError_t r2c_impl(const Dims& d, const double* in, cd* out, const cd* tw, hipStream_t s) {
    const long teams = (long)d.B * (N / 2);
    const int tpb = row_teams<N>(d, teams);
    hipLaunchKernelGGL(row_r2c_kernel<N>, dim3((unsigned)(teams / tpb)), dim3(tpb * Plan<N>::T),
                       row_lds<N>(tpb), s, d, in, out, tw);
    return hipGetLastError();
}
hipError_t launch_row_r2c(const Dims& d, const double* in, cd* out, const cd* tw, hipStream_t s) {
    if (!in || !out || !tw) return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return r2c_impl<NN>(d, in, out, tw, s));
    return hipSuccess;
}

template <int N>
static hipError_t c2r_impl(const Dims& d, const cd* in, double* out, const cd* tw, hipStream_t s) {
    const long teams = (long)d.B * (N / 2);
    const int tpb = row_teams<N>(d, teams);
    hipLaunchKernelGGL(row_c2r_kernel<N>, dim3((unsigned)(teams / tpb)), dim3(tpb * Plan<N>::T),
                       row_lds<N>(tpb), s, d, in, out, tw);
    return hipGetLastError();
}
hipError_t launch_row_c2r(const Dims& d, const cd* in, double* out, const cd* tw, hipStream_t s) {
    if (!in || !out || !tw) return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return c2r_impl<NN>(d, in, out, tw, s));
    return hipSuccess;
}

template <int N>
static hipError_t nl_impl(const Dims& d, const RowArgs& a, hipStream_t s) {
    const long teams = (long)d.B * N;
    const int tpb = row_teams<N>(d, teams);
    hipLaunchKernelGGL(row_nl_kernel<N>, dim3((unsigned)(teams / tpb)), dim3(tpb * Plan<N>::T),
                       row_lds<N>(tpb), s, d, a);
    return hipGetLastError();
}
hipError_t launch_row_nl(const Dims& d, const RowArgs& a, hipStream_t s) {
    if (!a.yin[0] || !a.yin[1] || !a.yin[2] || !a.yin[3] || !a.yout[0] || !a.tw || !obs_ok(a.obs))
        return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return nl_impl<NN>(d, a, s));
    return hipSuccess;
}

template <int N>
static hipError_t obs_impl(const Dims& d, const RowArgs& a, hipStream_t s) {
    const long teams = (long)d.B * a.obs.M;
    const int tpb = row_teams<N>(d, teams);
    hipLaunchKernelGGL(row_obs_kernel<N>, dim3((unsigned)(teams / tpb)), dim3(tpb * Plan<N>::T),
                       row_lds<N>(tpb), s, d, a);
    return hipGetLastError();
}
hipError_t launch_row_obs(const Dims& d, const RowArgs& a, hipStream_t s) {
    if (!a.yin[0] || !a.yin[1] || !a.tw || a.obs.slot < 0 || !obs_ok(a.obs)) return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return obs_impl<NN>(d, a, s));
    return hipSuccess;
}

template <int N>
static hipError_t adj_impl(const Dims& d, const RowArgs& a, hipStream_t s) {
    const long teams = (long)d.B * N;
    const int tpb = row_teams<N>(d, teams);
    hipLaunchKernelGGL(row_adj_kernel<N>, dim3((unsigned)(teams / tpb)), dim3(tpb * Plan<N>::T),
                       row_lds<N>(tpb), s, d, a);
    return hipGetLastError();
}
hipError_t launch_row_adj(const Dims& d, const RowArgs& a, hipStream_t s) {
    for (int i = 0; i < 5; ++i)
        if (!a.yin[i]) return hipErrorInvalidValue;
    for (int i = 0; i < 4; ++i)
        if (!a.yout[i]) return hipErrorInvalidValue;
    if (!a.tw || !obs_ok(a.obs)) return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return adj_impl<NN>(d, a, s));
    return hipSuccess;
}

template <int N>
static hipError_t src_impl(const Dims& d, const RowArgs& a, int impulse, hipStream_t s) {
    const long teams = (long)d.B * N;
    const int tpb = row_teams<N>(d, teams);
    hipLaunchKernelGGL(row_src_kernel<N>, dim3((unsigned)(teams / tpb)), dim3(tpb * Plan<N>::T),
                       row_lds<N>(tpb), s, d, a, impulse);
    return hipGetLastError();
}
hipError_t launch_row_src(const Dims& d, const RowArgs& a, int impulse, hipStream_t s) {
    if (!a.yout[0] || !a.yout[1] || !a.tw || (!impulse && (!a.yin[0] || !a.yin[1] || !obs_ok(a.obs))))
        return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return src_impl<NN>(d, a, impulse, s));
    return hipSuccess;
}

template <int N, int MODE>
static hipError_t col_mode(const Dims& d, const ColArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)(d.KXP / d.cb), (unsigned)d.B);
    const dim3 block((unsigned)(d.cb * Plan<N>::T));
    const size_t lds = (size_t)d.cb * lds_team<N>() * sizeof(cd);
    hipLaunchKernelGGL((col_kernel<N, MODE>), grid, block, lds, s, d, a);
    return hipGetLastError();
}

template <int N>
static hipError_t col_impl(const Dims& d, int mode, const ColArgs& a, hipStream_t s) {
    switch (mode) {
        case COL_INIT: return col_mode<N, COL_INIT>(d, a, s);
        case COL_A: return col_mode<N, COL_A>(d, a, s);
        case COL_B: return col_mode<N, COL_B>(d, a, s);
        case COL_C: return col_mode<N, COL_C>(d, a, s);
        case COL_D: return col_mode<N, COL_D>(d, a, s);
        case COL_FILTER: return col_mode<N, COL_FILTER>(d, a, s);
        case COL_FROM_STATE: return col_mode<N, COL_FROM_STATE>(d, a, s);
        case COL_ADJ_C: return col_mode<N, COL_ADJ_C>(d, a, s);
        case COL_ADJ_B: return col_mode<N, COL_ADJ_B>(d, a, s);
        case COL_ADJ_A: return col_mode<N, COL_ADJ_A>(d, a, s);
        case COL_ADJ_N: return col_mode<N, COL_ADJ_N>(d, a, s);
        case COL_ADJ_SRC: return col_mode<N, COL_ADJ_SRC>(d, a, s);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_col(const Dims& d, int mode, const ColArgs& a, hipStream_t s) {
    if (!col_ptrs_ok(mode, a)) return hipErrorInvalidValue;
    PA_DISPATCH_N(d.N, return col_impl<NN>(d, mode, a, s));
    return hipSuccess;
}

}  // namespace pa
