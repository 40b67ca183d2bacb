// Entry points shared between the translation units of the library (not
// exported).
#pragma once
#include <stdint.h>

#include "../../include/mr3.h"

// Solve `count` problems of one precision (32 or 64) given by per-problem
// device pointers: d[p], e[p] inputs, W[p] and Z[p] outputs (Z[p] may be
// null, and Z itself may be null for no vectors), ldz[p] leading dimensions.
// Host arrays; results as for mr3_solve_batched.  The arguments are assumed
// valid (callers check them).
// work, work_bytes: a work region as for the public entry points (NULL: the
// handle's pool).
__attribute__((visibility("hidden"))) int mr3_solve_ptrs(
    mr3_handle h, int precision, int64_t count, const int64_t* n, const void* const* d,
    const void* const* e, const mr3_range_desc* ranges, int64_t* m, void* const* W,
    void* const* Z, const int64_t* ldz, void* work, size_t work_bytes, void* stream);

// Copy the parameters set on handle `src` to `dst`.
__attribute__((visibility("hidden"))) void mr3_handle_copy_params(mr3_handle dst, mr3_handle src);

// Device of a handle.
__attribute__((visibility("hidden"))) int mr3_handle_device(mr3_handle h);

// Release the rocBLAS handle the dense entry points made for `h` (if any).
__attribute__((visibility("hidden"))) void mr3_dense_release(mr3_handle h);
