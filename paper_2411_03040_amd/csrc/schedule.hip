// Scheduling helpers of batched execution: per-origin cost for
// longest-first ordering, and order-preserving compaction of the work items
// of models that are still iterating.

#include <hipcub/hipcub.hpp>

#include "mgx_internal.h"

namespace mgx {

// Per-origin cost (trace records over all rays) for ordering batched work.
__global__ void k_origin_cost(int N, int R, const int64_t *off, int64_t *cost)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    cost[o] = off[(int64_t)o * R + R] - off[(int64_t)o * R];
}

hipError_t launch_origin_cost(int N, int R, const int64_t *off, int64_t *cost, hipStream_t s)
{
    k_origin_cost<<<(N + 255) / 256, 256, 0, s>>>(N, R, off, cost);
    return hipGetLastError();
}

namespace {
struct ItemActive {
    const int *active;
    __device__ __forceinline__ bool operator()(const int4 &w) const { return active[w.x] != 0; }
};
}  // namespace

hipError_t launch_compact_items(const int4 *in, int n, int4 *out, int *count, const int *active,
                                void **tmp, size_t *tmp_bytes, hipStream_t s)
{
    size_t need = 0;
    ItemActive op{active};
    hipError_t e = hipcub::DeviceSelect::If(nullptr, need, in, out, count, n, op, s);
    if (e != hipSuccess) return e;
    if (need > *tmp_bytes) {
        if (*tmp) (void)hipFree(*tmp);
        *tmp = nullptr;
        e = hipMalloc(tmp, need);
        if (e != hipSuccess) {
            *tmp_bytes = 0;
            return e;
        }
        *tmp_bytes = need;
    }
    return hipcub::DeviceSelect::If(*tmp, need, in, out, count, n, op, s);
}

}  // namespace mgx
