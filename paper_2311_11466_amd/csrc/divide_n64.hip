// The fused divide for N = 64 (256 threads per pattern).
#pragma clang fp contract(off)   // as in divide.hip: one rounding for every prologue mode
#include "divide_fused.hpp"

namespace pty {
PTY_DEFINE_FUSED(64, 256)
}  // namespace pty
