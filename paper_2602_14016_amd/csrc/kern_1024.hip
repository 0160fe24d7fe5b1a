// Row and column passes for N = 1024 (both FFT plan variants).
#include "kernels_impl.hpp"

namespace pa {
template struct Launch<1024>;
}  // namespace pa
