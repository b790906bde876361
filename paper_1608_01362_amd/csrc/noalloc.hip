// One PageRank iteration without any allocation: the iteration workspace of
// cagra_pagerank_iter lives in a file-scope device array instead of a caller
// buffer. For callers that cannot allocate device memory (code under graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
#include <mutex>

#include "common.h"

namespace cagra {

size_t ws_blk_bytes(int32_t V, int32_t nb);
size_t ws_item_bytes(const cagra_segments *seg);
size_t ws_slot_bytes(const cagra_segments *seg);
cagra_status launch_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                           void *partial, hipStream_t st);
cagra_status launch_merge_pr(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t seed,
                             int32_t contrib_type, const float *rank_in, const double *scalars_in,
                             const float *partial, float *rank_out, void *contrib_out, double *scalars_out, void *ws,
                             hipStream_t st);
cagra_status check_pagerank_args(const cagra_graph *g, const cagra_segments *seg, double damping,
                                 int32_t restart_vertex, int32_t contrib_type, const void *rank_in,
                                 const void *contrib_in, const void *scalars_in, const void *partial,
                                 const void *rank_out, const void *contrib_out, const void *scalars_out);

// The scratch memory: one copy per GPU, held until the process ends. Host
// code never uses this name as an address (on the host it is a stand-in
// symbol); it uses the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[CAGRA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
static cagra_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CAGRA_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(CAGRA_E_CAPACITY, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CAGRA_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CAGRA_OK;
}

}  // namespace cagra

using namespace cagra;

extern "C" {

size_t cagra_noalloc_scratch_bytes(void) { return CAGRA_NOALLOC_SCRATCH_BYTES; }

cagra_status cagra_pagerank_iter_noalloc(const cagra_graph *g, const cagra_segments *seg, double damping,
                                         int32_t restart_vertex, int32_t contrib_type, const float *rank_in,
                                         const void *contrib_in, const double *scalars_in, float *partial,
                                         float *rank_out, void *contrib_out, double *scalars_out,
                                         hipStream_t stream) {
    cagra_status s = check_pagerank_args(g, seg, damping, restart_vertex, contrib_type, rank_in, contrib_in,
                                         scalars_in, partial, rank_out, contrib_out, scalars_out);
    if (s != CAGRA_OK) return s;
    const size_t need = ws_blk_bytes(seg->V, seg->nb) + ws_item_bytes(seg) + ws_slot_bytes(seg) + 256;
    if (need > CAGRA_NOALLOC_SCRATCH_BYTES)
        return fail(CAGRA_E_CAPACITY,
                    "the iteration needs %zu bytes of scratch; the static scratch holds %zu (use "
                    "cagra_pagerank_iter with a workspace)",
                    need, (size_t)CAGRA_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((s = scratch_address(&ws)) != CAGRA_OK) return s;
    if ((s = launch_gather(seg, CAGRA_SUM_F32, contrib_type, contrib_in, partial, stream)) != CAGRA_OK) return s;
    return launch_merge_pr(g, seg, damping, restart_vertex, contrib_type, rank_in, scalars_in, partial, rank_out,
                           contrib_out, scalars_out, ws, stream);
}

}  // extern "C"
