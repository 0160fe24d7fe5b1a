// Row and column passes for N = 16 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<16>;
}  // namespace pa
