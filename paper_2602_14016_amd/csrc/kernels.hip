// kernels.hip -- dispatch of the row / column passes to the per-grid-size
// instantiations (kern_<N>.hip), with host-side argument checks so that a
// launch with a missing buffer is refused before it can touch memory.
#include "kernels.hpp"

namespace pa {

DispatchEvents& dispatch_events() {
    static thread_local DispatchEvents e;
    return e;
}

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
        case COL_FIRST_GUESS: return a.yin[0] && a.yin[1] && a.lowpass >= 0;
        case COL_ADJ_C: case COL_ADJ_B: case COL_ADJ_A: case COL_ADJ_N: case COL_ADJ_SRC: case COL_ADJ_NSRC:
            // extra (observation source) inputs are read by COL_ADJ_NSRC only
            if (a.nin < 2 || a.nin > (mode == COL_ADJ_NSRC ? 4 : 2) || !a.lam) return false;
            if (mode != COL_ADJ_SRC && !a.omb) return false;
            for (int p = 0; p < a.nin; ++p)
                if (!a.yin[p] || a.inmul[p] < IN_PAIRP || a.inmul[p] > IN_MIKX_INVK2) return false;
            return true;
        default: return false;
    }
}

#define PA_DISPATCH_N(CALL)                                   \
    switch (d.N) {                                            \
        case 8: return Launch<8>::CALL;                       \
        case 16: return Launch<16>::CALL;                     \
        case 32: return Launch<32>::CALL;                     \
        case 64: return Launch<64>::CALL;                     \
        case 128: return Launch<128>::CALL;                   \
        case 256: return Launch<256>::CALL;                   \
        case 512: return Launch<512>::CALL;                   \
        case 1024: return Launch<1024>::CALL;                 \
        default: return hipErrorInvalidValue;                 \
    }

int fft_threads(int N, int var) {
    switch (N) {
        case 8: return Launch<8>::threads(var);
        case 16: return Launch<16>::threads(var);
        case 32: return Launch<32>::threads(var);
        case 64: return Launch<64>::threads(var);
        case 128: return Launch<128>::threads(var);
        case 256: return Launch<256>::threads(var);
        case 512: return Launch<512>::threads(var);
        default: return Launch<1024>::threads(var);
    }
}

hipError_t launch_row_r2c(const Dims& d, const double* in, cd* out, const cd* tw, hipStream_t s) {
    if (!in || !out || !tw) return hipErrorInvalidValue;
    PA_DISPATCH_N(row_r2c(d, in, out, tw, s));
}
hipError_t launch_row_c2r(const Dims& d, const cd* in, double* out, const cd* tw, hipStream_t s) {
    if (!in || !out || !tw) return hipErrorInvalidValue;
    PA_DISPATCH_N(row_c2r(d, in, out, tw, s));
}
hipError_t launch_row_nl(const Dims& d, const RowArgs& a, hipStream_t s) {
    if (!a.yin[0] || !a.yin[1] || !a.yin[2] || !a.yin[3] || !a.yout[0] || !a.tw || !obs_ok(a.obs))
        return hipErrorInvalidValue;
    PA_DISPATCH_N(row_nl(d, a, s));
}
hipError_t launch_row_obs(const Dims& d, const RowArgs& a, hipStream_t s) {
    if (!a.yin[0] || !a.yin[1] || !a.yin[2] || !a.yin[3] || !a.tw || a.obs.slot < 0 || !obs_ok(a.obs))
        return hipErrorInvalidValue;
    PA_DISPATCH_N(row_obs(d, a, s));
}
hipError_t launch_row_adj(const Dims& d, const RowArgs& a, hipStream_t s) {
    for (int i = 0; i < 6; ++i)
        if (!a.yin[i]) return hipErrorInvalidValue;
    if (!a.yout[0] || !a.yout[1] || !a.tw) return hipErrorInvalidValue;
    PA_DISPATCH_N(row_adj(d, a, s));
}
hipError_t launch_row_src(const Dims& d, const RowArgs& a, int impulse, hipStream_t s) {
    if (!a.yout[0] || !a.yout[1] || !a.tw ||
        (!impulse && (!a.yin[0] || !a.yin[1] || !a.yin[2] || !a.yin[3] || !obs_ok(a.obs))))
        return hipErrorInvalidValue;
    PA_DISPATCH_N(row_src(d, a, impulse, s));
}
hipError_t launch_col(const Dims& d, int mode, const ColArgs& a, hipStream_t s) {
    if (!col_ptrs_ok(mode, a)) return hipErrorInvalidValue;
    PA_DISPATCH_N(col(d, mode, a, s));
}

}  // namespace pa
