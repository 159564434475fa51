// The fused divide for N = 32 (64 threads per pattern).
#include "divide_fused.hpp"

namespace pty {
PTY_DEFINE_FUSED(32, 64)
}  // namespace pty
