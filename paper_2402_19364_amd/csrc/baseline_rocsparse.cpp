// Comparison baseline: the vendor CSR SpMM (rocSPARSE generic API), y = A x
// with FP32 values, int32 indices and row-major dense matrices.  Only the
// benchmark calls it; the arrow path does not depend on it.
#include <hip/hip_runtime_api.h>
#include <rocsparse/rocsparse.h>

#include <new>
#include <string>

#include "arrow.h"
#include "internal.h"

struct arrow_rocsparse_s {
    rocsparse_handle handle = nullptr;
    rocsparse_spmat_descr a = nullptr;
    rocsparse_dnmat_descr x = nullptr, y = nullptr;
    void *buffer = nullptr;
    rocsparse_spmm_alg alg = rocsparse_spmm_alg_default;
};

namespace {

void release(arrow_rocsparse_s *c) {
    if (!c) return;
    if (c->buffer) hipFree(c->buffer);
    if (c->x) rocsparse_destroy_dnmat_descr(c->x);
    if (c->y) rocsparse_destroy_dnmat_descr(c->y);
    if (c->a) rocsparse_destroy_spmat_descr(c->a);
    if (c->handle) rocsparse_destroy_handle(c->handle);
    delete c;
}

arrow_status_t fail(arrow_rocsparse_s *c, const char *what, int code) {
    release(c);
    arrow::set_error(std::string("rocsparse: ") + what + " failed (" + std::to_string(code) + ")");
    return ARROW_ERR_HIP;
}

}  // namespace

extern "C" {

arrow_status_t arrow_rocsparse_create(int64_t n, int64_t nnz, const int32_t *row_ptr,
                                      const int32_t *col, const float *val, const float *x,
                                      float *y, int64_t k, int64_t ld, int32_t alg, void *stream,
                                      arrow_rocsparse_t *out) {
    if (!out || n <= 0 || k <= 0 || ld < k || !row_ptr || !x || !y || (nnz > 0 && (!col || !val))) {
        arrow::set_error("rocsparse baseline: bad arguments");
        return ARROW_ERR_INVALID_ARG;
    }
    *out = nullptr;
    auto *c = new (std::nothrow) arrow_rocsparse_s();
    if (!c) return ARROW_ERR_OUT_OF_MEMORY;
    c->alg = static_cast<rocsparse_spmm_alg>(alg);
    rocsparse_status s = rocsparse_create_handle(&c->handle);
    if (s != rocsparse_status_success) return fail(c, "create_handle", s);
    s = rocsparse_set_stream(c->handle, static_cast<hipStream_t>(stream));
    if (s != rocsparse_status_success) return fail(c, "set_stream", s);
    s = rocsparse_create_csr_descr(&c->a, n, n, nnz, const_cast<int32_t *>(row_ptr),
                                   const_cast<int32_t *>(col), const_cast<float *>(val),
                                   rocsparse_indextype_i32, rocsparse_indextype_i32,
                                   rocsparse_index_base_zero, rocsparse_datatype_f32_r);
    if (s != rocsparse_status_success) return fail(c, "create_csr_descr", s);
    s = rocsparse_create_dnmat_descr(&c->x, n, k, ld, const_cast<float *>(x),
                                     rocsparse_datatype_f32_r, rocsparse_order_row);
    if (s != rocsparse_status_success) return fail(c, "create_dnmat_descr", s);
    s = rocsparse_create_dnmat_descr(&c->y, n, k, ld, y, rocsparse_datatype_f32_r,
                                     rocsparse_order_row);
    if (s != rocsparse_status_success) return fail(c, "create_dnmat_descr", s);
    const float one = 1.0f, zero = 0.0f;
    size_t bytes = 0;
    s = rocsparse_spmm(c->handle, rocsparse_operation_none, rocsparse_operation_none, &one, c->a,
                       c->x, &zero, c->y, rocsparse_datatype_f32_r, c->alg,
                       rocsparse_spmm_stage_buffer_size, &bytes, nullptr);
    if (s != rocsparse_status_success) return fail(c, "spmm buffer_size", s);
    if (bytes > 0 && hipMalloc(&c->buffer, bytes) != hipSuccess) return fail(c, "hipMalloc", 0);
    s = rocsparse_spmm(c->handle, rocsparse_operation_none, rocsparse_operation_none, &one, c->a,
                       c->x, &zero, c->y, rocsparse_datatype_f32_r, c->alg,
                       rocsparse_spmm_stage_preprocess, &bytes, c->buffer);
    if (s != rocsparse_status_success) return fail(c, "spmm preprocess", s);
    *out = c;
    return ARROW_OK;
}

arrow_status_t arrow_rocsparse_run(arrow_rocsparse_t c) {
    if (!c) {
        arrow::set_error("rocsparse baseline: NULL context");
        return ARROW_ERR_INVALID_ARG;
    }
    const float one = 1.0f, zero = 0.0f;
    size_t bytes = 0;
    rocsparse_status s =
        rocsparse_spmm(c->handle, rocsparse_operation_none, rocsparse_operation_none, &one, c->a,
                       c->x, &zero, c->y, rocsparse_datatype_f32_r, c->alg,
                       rocsparse_spmm_stage_compute, &bytes, c->buffer);
    if (s != rocsparse_status_success) {
        arrow::set_error("rocsparse: spmm compute failed (" + std::to_string(s) + ")");
        return ARROW_ERR_HIP;
    }
    return ARROW_OK;
}

void arrow_rocsparse_destroy(arrow_rocsparse_t c) { release(c); }

}  // extern "C"
