// Frequency-based clustering (Section 5) and relabelling, before segmenting.
//
// 1. Vertex keys: out-degree where it is strictly above the average degree
//    E / V, else 0, stored bit-inverted so that a stable ascending radix sort
//    of (key, id) pairs gives the new order: clustered vertices by out-degree
//    from high to low (ties keep the original order), then every other vertex
//    in its original order.
// 2. inv[perm[i]] = i; new out-degrees and in-degrees follow perm; a scan of
//    the in-degrees gives the new row offsets.
// 3. Every edge u -> v becomes the key (inv[v] << b) | inv[u] (b bits per id);
//    one radix sort of these keys lays the edges out row by row with sources
//    ascending, and the low bits are the new source ids.
//
// The sorts are the stable radix passes of segsort.hip and the scan the
// builder's; clustering runs once per graph, off the iteration's hot path.
#include <cstring>

#include "common.h"

namespace cagra {

struct NoValue;
template <typename K, typename V>
cagra_status radix_sort_stable(const K *keys_in, const V *vals_in, K *keys_out, V *vals_out, int64_t n, int bits,
                               void *ws, size_t ws_bytes, hipStream_t st);
size_t sort_ws_bytes(int64_t n, int bits, int key_bytes, int value_bytes);
cagra_status scan_add_exclusive(const int32_t *in, int32_t *out, int64_t n, void *ws, size_t ws_bytes,
                                hipStream_t st);
size_t scan_add_ws_bytes(int64_t n);

constexpr int kEdgesPerThread = 16;

__global__ void k_cl_vertex_keys(const int32_t *__restrict__ outdeg, int32_t V, int64_t E,
                                 uint32_t *__restrict__ key, int32_t *__restrict__ id) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int64_t od = outdeg[v];
    key[v] = ~(od * (int64_t)V > E ? (uint32_t)od : 0u);
    id[v] = (int32_t)v;
}

// inv, the new out-degrees and in-degrees, and the clustered-vertex count.
__global__ void k_cl_relabel(const int32_t *__restrict__ perm, const uint32_t *__restrict__ key_sorted,
                             const int32_t *__restrict__ in_offsets, const int32_t *__restrict__ outdeg, int32_t V,
                             int32_t *__restrict__ inv, int32_t *__restrict__ outdeg_new, int32_t *__restrict__ cnt,
                             int32_t *__restrict__ hot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > V) return;
    if (i == V) {
        cnt[V] = 0;
        return;
    }
    const int32_t old = perm[i];
    inv[old] = (int32_t)i;
    outdeg_new[i] = outdeg[old];
    cnt[i] = in_offsets[old + 1] - in_offsets[old];
    if (hot) {
        // exactly one writer: the last clustered vertex, or vertex 0 when there is none
        // keys are stored bit-inverted: a clustered vertex has ~key > 0
        const bool last_hot = ~key_sorted[i] > 0u && (i + 1 == V || ~key_sorted[i + 1] == 0u);
        if (last_hot) *hot = (int32_t)(i + 1);
        if (i == 0 && ~key_sorted[0] == 0u) *hot = 0;
    }
}

// Last row r with in_offsets[r] <= e (the non-empty row holding edge e).
__device__ __forceinline__ int32_t row_of_edge(const int32_t *__restrict__ off, int32_t V, int64_t e) {
    int32_t lo = 0, hi = V;  // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)off[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Edge keys (new destination, new source) for a tile of kKeyThreads *
// kEdgesPerThread consecutive edges: the tile's sources are staged in LDS with
// coalesced loads, each thread takes kEdgesPerThread consecutive edges (the
// first one's row by binary search, then walking the offsets), and the keys
// leave through LDS with coalesced stores.
constexpr int kKeyThreads = 256;
constexpr int kKeyTile = kKeyThreads * kEdgesPerThread;

__global__ __launch_bounds__(kKeyThreads) void k_cl_edge_keys(const int32_t *__restrict__ in_offsets,
                                                              const int32_t *__restrict__ in_sources, int32_t V,
                                                              int64_t E, const int32_t *__restrict__ inv, int bits,
                                                              unsigned long long *__restrict__ keys) {
    __shared__ int32_t src[kKeyTile];
    __shared__ unsigned long long key[kKeyTile];
    const int64_t base = (int64_t)blockIdx.x * kKeyTile;
    const int n = (int)(E - base < kKeyTile ? E - base : kKeyTile);
    for (int i = threadIdx.x; i < n; i += kKeyThreads) src[i] = in_sources[base + i];
    __syncthreads();
    const int i0 = threadIdx.x * kEdgesPerThread;
    if (i0 < n) {
        const int i1 = i0 + kEdgesPerThread < n ? i0 + kEdgesPerThread : n;
        int32_t r = row_of_edge(in_offsets, V, base + i0);
        for (int i = i0; i < i1; ++i) {
            while ((int64_t)in_offsets[r + 1] <= base + i) ++r;
            key[i] = ((unsigned long long)(uint32_t)inv[r] << bits) | (unsigned long long)(uint32_t)inv[src[i]];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kKeyThreads) keys[base + i] = key[i];
}

__global__ void k_cl_sources(const unsigned long long *__restrict__ keys, int64_t E, unsigned long long mask,
                             int32_t *__restrict__ in_sources_new) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) in_sources_new[e] = (int32_t)(keys[e] & mask);
}

static int id_bits(int32_t V) {
    int b = 1;
    while (b < 31 && (1LL << b) < (int64_t)V) ++b;
    return b;
}

static unsigned grid_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Temporary-storage sizes of the two sorts and the scan.
struct ClusterTemps {
    size_t vsort = 0, scan = 0, esort = 0;
};

static cagra_status cluster_temps(int32_t V, int64_t E, ClusterTemps &t) {
    const int bits = id_bits(V);
    t.vsort = sort_ws_bytes(V, 32, 4, 4);
    t.scan = scan_add_ws_bytes((int64_t)V + 1);
    t.esort = E > 0 ? sort_ws_bytes(E, 2 * bits, 8, 0) : 0;
    return CAGRA_OK;
}

static size_t cluster_layout(int32_t V, int64_t E, const ClusterTemps &t) {
    ArenaSize a;
    a.take<uint32_t>(V);                 // key
    a.take<uint32_t>(V);                 // key_sorted
    a.take<int32_t>(V);                  // id
    a.take<int32_t>(V);                  // inv
    a.take<int32_t>((int64_t)V + 1);     // cnt
    a.take<unsigned long long>(E);       // edge keys
    a.take<unsigned long long>(E);       // sorted edge keys
    size_t tmp = t.vsort > t.scan ? t.vsort : t.scan;
    if (t.esort > tmp) tmp = t.esort;
    a.take<char>((int64_t)tmp);
    return a.used + 256;
}

cagra_status cluster_workspace_bytes(int32_t V, int64_t E, size_t *bytes) {
    ClusterTemps t;
    if (cagra_status s = cluster_temps(V, E, t)) return s;
    *bytes = cluster_layout(V, E, t);
    return CAGRA_OK;
}

cagra_status cluster_graph(const cagra_graph *g, int32_t *perm, int32_t *in_offsets_new, int32_t *in_sources_new,
                           int32_t *outdeg_new, int32_t *hot, void *ws, size_t ws_bytes, hipStream_t st) {
    const int32_t V = g->V;
    const int64_t E = g->E;
    ClusterTemps t;
    if (cagra_status s = cluster_temps(V, E, t)) return s;
    const size_t need = cluster_layout(V, E, t);
    if (ws_bytes < need) return fail(CAGRA_E_BUFFER, "cluster workspace needs %zu bytes (got %zu)", need, ws_bytes);
    Arena ar{(char *)ws, ws_bytes, 0};
    uint32_t *key = ar.take<uint32_t>(V);
    uint32_t *key_sorted = ar.take<uint32_t>(V);
    int32_t *id = ar.take<int32_t>(V);
    int32_t *inv = ar.take<int32_t>(V);
    int32_t *cnt = ar.take<int32_t>((int64_t)V + 1);
    unsigned long long *ekeys = ar.take<unsigned long long>(E);
    unsigned long long *ekeys_sorted = ar.take<unsigned long long>(E);
    size_t tmp_bytes = t.vsort > t.scan ? t.vsort : t.scan;
    if (t.esort > tmp_bytes) tmp_bytes = t.esort;
    char *tmp = ar.take<char>((int64_t)tmp_bytes);
    if (!key || !key_sorted || !id || !inv || !cnt || !ekeys || !ekeys_sorted || !tmp)
        return fail(CAGRA_E_BUFFER, "cluster workspace smaller than %zu bytes", need);

    // 1. new vertex order
    k_cl_vertex_keys<<<grid_of(V, 256), 256, 0, st>>>(g->out_degree, V, E, key, id);
    CAGRA_LAUNCH_CHECK();
    cagra_status s;
    if ((s = radix_sort_stable<uint32_t, int32_t>(key, id, key_sorted, perm, V, 32, tmp, tmp_bytes, st)) != CAGRA_OK)
        return s;
    // 2. relabel vertices, new row offsets
    k_cl_relabel<<<grid_of((int64_t)V + 1, 256), 256, 0, st>>>(perm, key_sorted, g->in_offsets, g->out_degree, V,
                                                                inv, outdeg_new, cnt, hot);
    CAGRA_LAUNCH_CHECK();
    if ((s = scan_add_exclusive(cnt, in_offsets_new, (int64_t)V + 1, tmp, tmp_bytes, st)) != CAGRA_OK) return s;
    if (E == 0) return CAGRA_OK;
    // 3. relabel edges: one sort by (new destination, new source)
    const int bits = id_bits(V);
    k_cl_edge_keys<<<grid_of(E, kKeyTile), kKeyThreads, 0, st>>>(g->in_offsets, g->in_sources, V, E, inv, bits,
                                                                 ekeys);
    CAGRA_LAUNCH_CHECK();
    if ((s = radix_sort_stable<unsigned long long, NoValue>(ekeys, nullptr, ekeys_sorted, nullptr, E, 2 * bits, tmp,
                                                             tmp_bytes, st)) != CAGRA_OK)
        return s;
    k_cl_sources<<<grid_of(E, 256), 256, 0, st>>>(ekeys_sorted, E, (1ull << bits) - 1ull, in_sources_new);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
