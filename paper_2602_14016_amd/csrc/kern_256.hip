// Row and column passes for N = 256 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<256>;
}  // namespace pa
