// The fused divide for N = 128 (512 threads per pattern).
#include "divide_fused.hpp"

namespace pty {
PTY_DEFINE_FUSED(128, 512)
}  // namespace pty
