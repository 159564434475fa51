// The fused divide for N = 64 (256 threads per pattern).
#include "divide_fused.hpp"

namespace pty {
PTY_DEFINE_FUSED(64, 256)
}  // namespace pty
