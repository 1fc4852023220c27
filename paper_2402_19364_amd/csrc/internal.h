// Internal declarations shared by the host sources of libarrow.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "arrow.h"

namespace arrow {

// One level of the decomposition: B_i over positions [0, n_i) and the vertex at
// each position.
struct Level {
    int64_t n_i = 0;
    std::vector<int32_t> vop;      // vertex of position, [n_i]
    std::vector<int64_t> row_ptr;  // [n_i + 1]
    std::vector<int32_t> col;      // positions, sorted within a row
    std::vector<float> val;
};

struct Decomp {
    int64_t n = 0, nnz = 0;
    int32_t b = 0;
    int32_t la = 0;
    uint64_t seed = 0;
    double seconds = 0.0;
    std::vector<Level> levels;
};

// Thread-local error text (set by the functions below on failure).
void set_error(const std::string &msg);

// Validates the CSR and runs LA-Decompose.  Returns ARROW_OK or an error code.
arrow_status_t decompose(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const float *val, const arrow_decompose_opts_t &opts, Decomp &out);

// Device of a plan handle.
int plan_device(arrow_plan_t p);

arrow_status_t save_decomp(const Decomp &d, const char *path);
arrow_status_t load_decomp(const char *path, Decomp &out);

}  // namespace arrow
