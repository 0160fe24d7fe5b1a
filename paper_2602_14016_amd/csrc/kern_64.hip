// Row and column passes for N = 64 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<64>;
}  // namespace pa
