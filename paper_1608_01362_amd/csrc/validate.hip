// Device check of the in-edge CSC that every entry point assumes: offsets that
// start at 0, end at E and never decrease; sources in [0, V), strictly
// ascending within each row (no duplicates) and never equal to the row (no
// self-loops). Two passes: the offsets first, then - only when they are sound,
// so that every read stays inside the arrays - the edges, each finding its row
// by binary search. Each violation class sets a bit and records its smallest
// index, so the report names the first offending vertex or edge.
#include "common.h"

namespace cagra {

constexpr int kValThreads = 256;

// report[0]: violation bits; report[1 + c]: smallest index of class c
enum : uint32_t {
    kBadFirst = 1u << 0,    // in_offsets[0] != 0
    kBadLast = 1u << 1,     // in_offsets[V] != E
    kDecreasing = 1u << 2,  // in_offsets[v + 1] < in_offsets[v]
    kRange = 1u << 3,       // source outside [0, V)
    kOrder = 1u << 4,       // sources not strictly ascending in a row
    kSelf = 1u << 5,        // self-loop
};
constexpr int kClasses = 6;

__device__ __forceinline__ void report_at(unsigned long long *rep, int cls, int64_t idx) {
    atomicOr(&rep[0], 1ull << cls);
    atomicMin(&rep[1 + cls], (unsigned long long)idx);
}

__global__ void k_val_init(unsigned long long *rep) {
    if (threadIdx.x == 0) rep[0] = 0ull;
    if (threadIdx.x < kClasses) rep[1 + threadIdx.x] = ~0ull;
}

__global__ __launch_bounds__(kValThreads) void k_val_offsets(const int32_t *__restrict__ off, int32_t V, int64_t E,
                                                             unsigned long long *__restrict__ rep) {
    const int64_t v = (int64_t)blockIdx.x * kValThreads + threadIdx.x;
    if (v == 0 && off[0] != 0) report_at(rep, 0, 0);
    if (v == 0 && (int64_t)off[V] != E) report_at(rep, 1, V);
    if (v < V && off[v + 1] < off[v]) report_at(rep, 2, v);
}

// Row of edge e: the last v with off[v] <= e (offsets already checked).
__device__ __forceinline__ int32_t val_row_of(const int32_t *__restrict__ off, int32_t V, int64_t e) {
    int32_t lo = 0, hi = V;
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)off[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kValThreads) void k_val_edges(const int32_t *__restrict__ off,
                                                           const int32_t *__restrict__ src, int32_t V, int64_t E,
                                                           unsigned long long *__restrict__ rep) {
    const int64_t e = (int64_t)blockIdx.x * kValThreads + threadIdx.x;
    if (e >= E) return;
    const int32_t u = src[e];
    if (u < 0 || u >= V) report_at(rep, 3, e);
    const int32_t v = val_row_of(off, V, e);
    if (u == v) report_at(rep, 5, e);
    if ((int64_t)off[v] < e && src[e - 1] >= u) report_at(rep, 4, e);
}

static const char *kClassText[kClasses] = {
    "in_offsets[0] is not 0", "in_offsets[V] is not E", "in_offsets decreases at vertex",
    "source out of range at edge", "sources not strictly ascending (or duplicated) at edge", "self-loop at edge"};

size_t validate_ws_bytes() { return 256; }

static cagra_status read_report(unsigned long long *rep, hipStream_t st, unsigned long long *host) {
    CAGRA_HIP_CHECK(hipMemcpyAsync(host, rep, sizeof(unsigned long long) * (1 + kClasses), hipMemcpyDeviceToHost,
                                   st));
    CAGRA_HIP_CHECK(hipStreamSynchronize(st));
    return CAGRA_OK;
}

static cagra_status report_status(const unsigned long long *host) {
    for (int c = 0; c < kClasses; ++c)
        if (host[0] & (1ull << c))
            return fail(CAGRA_E_INVALID, "graph check: %s %llu", kClassText[c], (unsigned long long)host[1 + c]);
    return CAGRA_OK;
}

cagra_status validate_graph(const cagra_graph *g, void *ws, hipStream_t st) {
    unsigned long long *rep = static_cast<unsigned long long *>(ws);
    unsigned long long host[1 + kClasses];
    k_val_init<<<1, 64, 0, st>>>(rep);
    CAGRA_LAUNCH_CHECK();
    k_val_offsets<<<(unsigned)ceil_div((int64_t)g->V + 1, kValThreads), kValThreads, 0, st>>>(g->in_offsets, g->V,
                                                                                             g->E, rep);
    CAGRA_LAUNCH_CHECK();
    if (cagra_status s = read_report(rep, st, host)) return s;
    if (cagra_status s = report_status(host)) return s;
    if (g->E > 0) {
        k_val_edges<<<(unsigned)ceil_div(g->E, kValThreads), kValThreads, 0, st>>>(g->in_offsets, g->in_sources,
                                                                                   g->V, g->E, rep);
        CAGRA_LAUNCH_CHECK();
        if (cagra_status s = read_report(rep, st, host)) return s;
        if (cagra_status s = report_status(host)) return s;
    }
    return CAGRA_OK;
}

}  // namespace cagra
