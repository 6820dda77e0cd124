// Graph preparation for the bottom-up BFS levels (run once, when a graph
// is wrapped): a library-owned copy of the column array in which every
// vertex's neighbours are ordered by decreasing degree, ties in their
// original order.
//
// A bottom-up level asks, for every unvisited vertex, whether any
// neighbour is in the current frontier, and stops at the first one found.
// On power-law graphs the frontier of the large bottom-up levels holds the
// high-degree vertices first, so a list that starts with its highest-degree
// neighbours mostly answers on its first arc: on R-MAT scale 22 the first
// arc already decides 92% of the vertices found at the largest bottom-up
// level, against 36% in id order, and 0.5% instead of 22% need more than
// one 4-arc probe. The order only changes which arc answers first, never
// the answer, so levels are unchanged.
//
// The order is computed with rocPRIM's stable segmented radix sort (one
// segment per vertex): keys are the neighbours' degrees, values the
// neighbour ids. The copy holds 4 padding words after the last arc, so that
// a probe may load the aligned 16 bytes that hold any arc.
//
// On a skewed graph (a maximum degree above 16 times the average), every
// vertex's first two neighbours in that order also sit in a dense array (8
// bytes per vertex): the first probe of a bottom-up candidate reads them,
// and since the candidates of a block are consecutive vertices, a block's
// first probes share cache lines instead of fetching one line of the column
// array each (on R-MAT 22 the largest bottom-up level fetched about 300 MB
// that way, one 128-byte line per candidate; with the dense array a
// 10-source launch runs 5% faster). On a graph without hubs the first two
// arcs decide too few candidates for that: most would then need a second
// round, so the dense read adds an access instead of replacing one (the
// 512-instance ER batch ran 12% slower), and no array is built.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "coop_internal.h"

namespace {

// key of arc e = degree of its head (the neighbour), from row_ptr
__global__ void neighbour_degree_kernel(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ col,
                                        uint64_t arcs, uint32_t* __restrict__ key) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < arcs;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = col[e];
        key[e] = row_ptr[u + 1] - row_ptr[u];
    }
}

__global__ void first_two_kernel(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ col_bu,
                                 uint32_t n, uint2* __restrict__ first2) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t a = row_ptr[v], d = row_ptr[v + 1] - a;
        first2[v] = make_uint2(d > 0 ? col_bu[a] : 0xFFFFFFFFu, d > 1 ? col_bu[a + 1] : 0xFFFFFFFFu);
    }
}

uint32_t bits_for(uint32_t max_value) {
    uint32_t b = 1;
    while (b < 32 && (max_value >> b) != 0) ++b;
    return b;
}

}  // namespace

namespace coop {

// Sorted copy of `col` into `out` (arcs + 4 words, caller-allocated):
// allocates and frees its own temporaries on `s` and waits for the stream.
hipError_t build_degree_order(const uint32_t* row_ptr, const uint32_t* col, uint32_t n, uint64_t arcs,
                              uint32_t max_deg, uint32_t* out, hipStream_t s) {
    if (arcs == 0) return hipMemsetAsync(out, 0, 16, s);
    if (arcs > 0xFFFFFFFFull) return hipErrorInvalidValue;
    uint32_t *key_in = nullptr, *key_out = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    hipError_t e = hipMalloc(&key_in, arcs * 4);
    if (e == hipSuccess) e = hipMalloc(&key_out, arcs * 4);
    if (e == hipSuccess) {
        uint64_t blocks = (arcs + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(neighbour_degree_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, row_ptr, col, arcs,
                           key_in);
        e = hipGetLastError();
    }
    const uint32_t end_bit = bits_for(max_deg);
    if (e == hipSuccess)
        e = rocprim::segmented_radix_sort_pairs_desc(nullptr, temp_bytes, key_in, key_out, col, out,
                                                     (unsigned int)arcs, n, row_ptr, row_ptr + 1, 0u, end_bit, s);
    if (e == hipSuccess) e = hipMalloc(&temp, temp_bytes ? temp_bytes : 4);
    if (e == hipSuccess)
        e = rocprim::segmented_radix_sort_pairs_desc(temp, temp_bytes, key_in, key_out, col, out,
                                                     (unsigned int)arcs, n, row_ptr, row_ptr + 1, 0u, end_bit, s);
    if (e == hipSuccess) e = hipMemsetAsync(out + arcs, 0, 16, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (temp) (void)hipFree(temp);
    if (key_out) (void)hipFree(key_out);
    if (key_in) (void)hipFree(key_in);
    return e;
}

hipError_t build_first_two(const uint32_t* row_ptr, const uint32_t* col_bu, uint32_t n, uint2* first2,
                           hipStream_t s) {
    uint32_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(first_two_kernel, dim3(blocks ? blocks : 1), dim3(256), 0, s, row_ptr, col_bu, n, first2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

}  // namespace coop
