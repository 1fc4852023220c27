// Row, chunk and permutation kernels stored as f32 (one translation unit per
// storage type, so the library builds in parallel).
#include "kernels_dev.h"

namespace arrow {
ARROW_INSTANTIATE_DT(kF32)
}  // namespace arrow
