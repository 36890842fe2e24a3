// limits.hpp -- constants shared by the host code and the kernels.
#pragma once

namespace rc {
// levels of the per-light triangle bins (B / 4^k bins per face side)
constexpr int kLbMaxLevels = 4;
}  // namespace rc
