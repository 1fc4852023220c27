// Row, chunk and permutation kernels stored as f8e4m3 (one translation unit per
// storage type, so the library builds in parallel).
#include "kernels_dev.h"

namespace arrow {
ARROW_INSTANTIATE_DT(kF8E4M3)
}  // namespace arrow
