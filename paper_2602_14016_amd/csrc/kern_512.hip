// Row and column passes for N = 512 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<512>;
}  // namespace pa
