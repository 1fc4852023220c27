// Row, chunk and permutation kernels stored as f16 (one translation unit per
// storage type, so the library builds in parallel).
#include "kernels_dev.h"

namespace arrow {
ARROW_INSTANTIATE_DT(kF16)
}  // namespace arrow
