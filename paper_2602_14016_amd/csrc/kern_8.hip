// Row and column passes for N = 8 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<8>;
}  // namespace pa
