// Row and column passes for N = 128 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<128>;
}  // namespace pa
