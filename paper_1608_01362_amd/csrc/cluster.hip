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
//    ascending, and its last pass writes the low bits, the new source ids.
//    The kernel that makes the keys also counts the first pass's digits.
//
// The sorts are the stable radix passes of segsort.hip and the scan the
// builder's; clustering runs once per graph, off the iteration's hot path.
#include <cstring>

#include "common.h"
#include "radix.h"

namespace cagra {

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

// Edge keys (new destination, new source) for a tile of kKeyTile consecutive
// edges, edge j * kKeyThreads + thread of the tile in step j (coalesced loads
// and stores). The tile's first row is found by a cooperative search (every
// round the workgroup probes kKeyThreads evenly spaced rows, so the interval
// shrinks by that factor); then the offsets of the rows the tile spans are
// staged in LDS a window of kOffWin rows at a time, and each edge finds its
// row by binary search in the window. The tile is also a tile of the sort, so
// the kernel publishes the counts of the sort's first digit (the low dbits0
// bits): counts0[d * gridDim.x + tile].
constexpr int kKeyThreads = 256;
constexpr int kKeyTile = kKeyThreads * kEdgesPerThread;
constexpr int kOffWin = 4096;
constexpr int kMaxDigits0 = 256;
static_assert(kKeyTile == kRadixTile, "key tiles are the sort's tiles");

__global__ __launch_bounds__(kKeyThreads) void k_cl_edge_keys(const int32_t *__restrict__ in_offsets,
                                                              const int32_t *__restrict__ in_sources, int32_t V,
                                                              int64_t E, const int32_t *__restrict__ inv, int bits,
                                                              int dbits0, unsigned long long *__restrict__ keys,
                                                              int32_t *__restrict__ counts0) {
    __shared__ int32_t off[kOffWin + 1];
    __shared__ int32_t nle[kKeyThreads / 64];
    __shared__ int32_t h[kMaxDigits0];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ndig = 1 << dbits0;
    for (int d = tid; d < ndig; d += kKeyThreads) h[d] = 0;  // ordered by the window loop's barriers
    const int tile = xcd_remap(blockIdx.x, gridDim.x);  // consecutive tiles on one XCD, as in the sort
    const int64_t base = (int64_t)tile * kKeyTile;
    const int n = (int)(E - base < kKeyTile ? E - base : kKeyTile);
    const int64_t last = base + n - 1;
    // Loads are issued in batches and without branches (lanes past the end
    // read the tile's last edge), so that their latencies overlap: the
    // sources now, the offset windows and the new ids further down.
    int32_t src[kEdgesPerThread];
#pragma unroll
    for (int j = 0; j < kEdgesPerThread; ++j) {
        const int64_t e = base + j * kKeyThreads + tid;
        src[j] = in_sources[e <= last ? e : last];
    }
    // first row: the last r with in_offsets[r] <= base (in_offsets[0] = 0 <= base < E = in_offsets[V])
    int32_t lo = 0, hi = V;  // in_offsets[lo] <= base < in_offsets[hi]
    while (hi - lo > 1) {
        const int32_t m = lo + (int32_t)(((int64_t)(hi - lo) * tid) / kKeyThreads);  // m = lo for thread 0
        const bool le = (int64_t)in_offsets[m] <= base;
        const uint64_t bal = __ballot(le);
        if (lane == 0) nle[w] = (int32_t)__popcll(bal);
        __syncthreads();
        int32_t t = -1;
        for (int x = 0; x < kKeyThreads / 64; ++x) t += nle[x];
        __syncthreads();
        // probes are non-decreasing in the thread index, so exactly threads 0..t found in_offsets <= base
        const int32_t nlo = lo + (int32_t)(((int64_t)(hi - lo) * t) / kKeyThreads);
        const int32_t nhi = t + 1 < kKeyThreads ? lo + (int32_t)(((int64_t)(hi - lo) * (t + 1)) / kKeyThreads) : hi;
        lo = nlo;
        hi = nhi;
    }
    int32_t rw = lo;  // first row of the window
    int32_t row[kEdgesPerThread] = {};
    static_assert(kOffWin % kKeyThreads == 0, "window staged in whole rounds");
    for (;;) {
        int32_t o[kOffWin / kKeyThreads];
#pragma unroll
        for (int k = 0; k < kOffWin / kKeyThreads; ++k) {
            const int64_t r = (int64_t)rw + k * kKeyThreads + tid;
            o[k] = in_offsets[r < V ? r : V];
        }
        const int64_t rend = (int64_t)rw + kOffWin;
        const int32_t oend = in_offsets[rend < V ? rend : V];
#pragma unroll
        for (int k = 0; k < kOffWin / kKeyThreads; ++k) off[k * kKeyThreads + tid] = o[k];
        if (tid == 0) off[kOffWin] = oend;
        __syncthreads();
        const int64_t wend = off[kOffWin];  // first edge past the window
#pragma unroll
        for (int j = 0; j < kEdgesPerThread; ++j) {
            const int64_t e = base + j * kKeyThreads + tid;
            if (e <= last && (int64_t)off[0] <= e && e < wend) {
                int a = 0, b = kOffWin;  // off[a] <= e < off[b]
                while (b - a > 1) {
                    const int mid = (a + b) >> 1;
                    if ((int64_t)off[mid] <= e) a = mid;
                    else b = mid;
                }
                row[j] = rw + a;
            }
        }
        __syncthreads();
        if (wend > last) break;
        rw += kOffWin;
    }
    // new ids (row[j] stays 0 for lanes past the end)
    uint32_t nd[kEdgesPerThread], ns[kEdgesPerThread];
#pragma unroll
    for (int j = 0; j < kEdgesPerThread; ++j) {
        nd[j] = (uint32_t)inv[row[j]];
        ns[j] = (uint32_t)inv[src[j]];
    }
#pragma unroll
    for (int j = 0; j < kEdgesPerThread; ++j) {
        const int64_t e = base + j * kKeyThreads + tid;
        if (e <= last) {
            const unsigned long long key = ((unsigned long long)nd[j] << bits) | (unsigned long long)ns[j];
            keys[e] = key;
            atomicAdd(&h[(int)(key & (unsigned long long)(ndig - 1))], 1);
        }
    }
    __syncthreads();
    for (int d = tid; d < ndig; d += kKeyThreads) counts0[(int64_t)d * gridDim.x + tile] = h[d];
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
    int64_t ncounts0 = 0;  // first-pass digit counts of the edge sort
};

static cagra_status cluster_temps(int32_t V, int64_t E, ClusterTemps &t) {
    const int bits = id_bits(V);
    t.vsort = sort_ws_bytes(V, 32, 4, 4);
    t.scan = scan_add_ws_bytes((int64_t)V + 1);
    t.esort = E > 0 ? sort_low32_ws_bytes(E, 2 * bits) : 0;
    t.ncounts0 = E > 0 ? ((int64_t)1 << sort_digit_bits(2 * bits)) * ceil_div(E, kKeyTile) : 0;
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
    a.take<unsigned long long>(E);       // edge keys between sort passes
    a.take<int32_t>(t.ncounts0);         // first-pass digit counts
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
    unsigned long long *ekeys_tmp = ar.take<unsigned long long>(E);
    int32_t *counts0 = ar.take<int32_t>(t.ncounts0);
    size_t tmp_bytes = t.vsort > t.scan ? t.vsort : t.scan;
    if (t.esort > tmp_bytes) tmp_bytes = t.esort;
    char *tmp = ar.take<char>((int64_t)tmp_bytes);
    if (!key || !key_sorted || !id || !inv || !cnt || !tmp || (E > 0 && (!ekeys || !ekeys_tmp || !counts0)))
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
    // 3. relabel edges: one sort by (new destination, new source); its last
    //    pass writes the new source ids
    const int bits = id_bits(V);
    const int dbits0 = sort_digit_bits(2 * bits);
    if (dbits0 > 8) return fail(CAGRA_E_CAPACITY, "first sort digit wider than the key kernel's count table");
    k_cl_edge_keys<<<grid_of(E, kKeyTile), kKeyThreads, 0, st>>>(g->in_offsets, g->in_sources, V, E, inv, bits,
                                                                 dbits0, ekeys, counts0);
    CAGRA_LAUNCH_CHECK();
    return radix_sort_low32(ekeys, ekeys_tmp, counts0, in_sources_new, E, 2 * bits, bits, tmp, tmp_bytes, st);
}

}  // namespace cagra
