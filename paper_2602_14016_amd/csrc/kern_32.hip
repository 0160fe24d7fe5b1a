// Row and column passes for N = 32 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<32>;
}  // namespace pa
