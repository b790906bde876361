// Many independent graphs in one launch per kernel: per-graph descriptors in
// device memory, global tile and merge-block lists, and persistent workgroups
// striding over them. A PageRank iteration of every graph is three kernel
// launches with no host synchronization, so a whole run can be captured into
// one HIP graph.
#include <vector>

#include "common.h"

namespace cagra {

cagra_status fail(cagra_status st, const char *fmt, ...);
size_t merge_fused_lds_total(int32_t B, int32_t k, int acc_bytes);
size_t merge_fused_lds_bytes(int32_t B, int32_t k, int acc_bytes);
cagra_status launch_multi_gather(const MultiDesc *desc, const int32_t *tile_graph, int64_t total_tiles, int parity,
                                 int grid, hipStream_t st);
cagra_status launch_multi_merge(const MultiDesc *desc, const int32_t *block_graph, int64_t total_blocks,
                                int32_t ngraphs, int parity, double damping, double *blk, size_t lds, int grid,
                                hipStream_t st);
cagra_status launch_multi_start(const MultiDesc *desc, const int32_t *block_graph, int64_t total_blocks,
                                int32_t ngraphs, double *blk, int grid, hipStream_t st);

static size_t desc_area(int32_t ngraphs) { return align_up((size_t)ngraphs * sizeof(MultiDesc), 256); }

static cagra_status check_multi_member(const cagra_graph *g, const cagra_segments *s, int i) {
    if (!g || !s) return fail(CAGRA_E_INVALID, "graph/segments %d is NULL", i);
    if (g->V < 1 || !g->in_offsets || !g->out_degree || (g->E > 0 && !g->in_sources))
        return fail(CAGRA_E_INVALID, "graph %d is incomplete", i);
    if (s->V != g->V || s->E != g->E || s->k != (int32_t)ceil_div(s->V, s->N) ||
        s->nb != (int32_t)ceil_div(s->V, s->B) || s->Q < 0 || s->Q > s->E || s->ntiles < 0)
        return fail(CAGRA_E_INVALID, "segments %d are inconsistent with graph %d", i, i);
    if (!s->seg_row_begin || !s->row_ptr || !s->row_dst || !s->edge_src || !s->block_ptr || !s->tile_edge ||
        !s->tile_seg || !s->tile_span_row || !s->row_dst_lo)
        return fail(CAGRA_E_INVALID, "a segments array of graph %d is NULL", i);
    if (((uintptr_t)s->edge_src & 15) != 0) return fail(CAGRA_E_INVALID, "edge_src of graph %d is misaligned", i);
    if ((size_t)s->N * 4 > CAGRA_STAGE_BYTES)
        return fail(CAGRA_E_CAPACITY, "graph %d: N=%d is not LDS-staged (multi-graph runs need N*4 <= %d)", i, s->N,
                    CAGRA_STAGE_BYTES);
    if (merge_fused_lds_total(s->B, s->k, 8) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "graph %d: B=%d with k=%d exceeds the merge LDS", i, s->B, s->k);
    return CAGRA_OK;
}

}  // namespace cagra

using namespace cagra;

extern "C" {

cagra_status cagra_multi_query(int32_t ngraphs, const cagra_graph *graphs, const cagra_segments *segs,
                               cagra_multi *m) {
    if (ngraphs < 1 || !graphs || !segs || !m) return fail(CAGRA_E_INVALID, "bad multi-graph arguments");
    int64_t V = 0, Q = 0, T = 0, Bk = 0;
    int32_t max_k = 0, max_B = 0;
    for (int32_t i = 0; i < ngraphs; ++i) {
        cagra_status s = check_multi_member(&graphs[i], &segs[i], i);
        if (s != CAGRA_OK) return s;
        V += graphs[i].V;
        Q += segs[i].Q;
        T += segs[i].ntiles;
        Bk += segs[i].nb;
        if (segs[i].k > max_k) max_k = segs[i].k;
        if (segs[i].B > max_B) max_B = segs[i].B;
    }
    if (T > INT32_MAX || Bk > INT32_MAX) return fail(CAGRA_E_OVERFLOW, "too many tiles or blocks");
    m->ngraphs = ngraphs;
    m->total_V = V;
    m->total_Q = Q;
    m->total_tiles = T;
    m->total_blocks = Bk;
    m->max_k = max_k;
    m->max_B = max_B;
    m->desc_bytes = desc_area(ngraphs) + (size_t)(T + Bk + 2) * sizeof(int32_t) + 256;
    return CAGRA_OK;
}

cagra_status cagra_multi_setup(cagra_multi *m, const cagra_graph *graphs, const cagra_segments *segs,
                               hipStream_t stream) {
    if (!m || !graphs || !segs || m->ngraphs < 1) return fail(CAGRA_E_INVALID, "bad multi-graph arguments");
    if (!m->desc || !m->rank[0] || !m->rank[1] || !m->contrib[0] || !m->contrib[1] || !m->scalars[0] ||
        !m->scalars[1] || !m->blk || (m->total_Q > 0 && !m->partial))
        return fail(CAGRA_E_INVALID, "a multi-graph pool is NULL");
    cagra_multi chk = *m;
    cagra_status s = cagra_multi_query(m->ngraphs, graphs, segs, &chk);
    if (s != CAGRA_OK) return s;
    if (chk.total_V != m->total_V || chk.total_Q != m->total_Q || chk.total_tiles != m->total_tiles ||
        chk.total_blocks != m->total_blocks || chk.desc_bytes != m->desc_bytes)
        return fail(CAGRA_E_INVALID, "graphs changed since cagra_multi_query");
    const int32_t n = m->ngraphs;
    std::vector<unsigned char> host(m->desc_bytes, 0);
    MultiDesc *d = reinterpret_cast<MultiDesc *>(host.data());
    int32_t *tile_graph = reinterpret_cast<int32_t *>(host.data() + desc_area(n));
    int32_t *block_graph = tile_graph + m->total_tiles;
    int64_t voff = 0, qoff = 0, tb = 0, bb = 0;
    for (int32_t i = 0; i < n; ++i) {
        const cagra_graph &g = graphs[i];
        const cagra_segments &sg = segs[i];
        MultiDesc &x = d[i];
        x.edge_src = sg.edge_src;
        x.tile_edge = sg.tile_edge;
        x.tile_seg = sg.tile_seg;
        x.tile_span_row = sg.tile_span_row;
        x.row_dst_lo = sg.row_dst_lo;
        x.block_ptr = sg.block_ptr;
        x.out_degree = g.out_degree;
        for (int p = 0; p < 2; ++p) {
            x.rank[p] = m->rank[p] + voff;
            x.contrib[p] = m->contrib[p] + voff;
            x.scalars[p] = m->scalars[p] + 4 * (int64_t)i;
        }
        x.partial = m->partial + qoff;
        x.Q = sg.Q;
        x.tile_base = tb;
        x.block_base = bb;
        x.V = g.V;
        x.N = sg.N;
        x.k = sg.k;
        x.B = sg.B;
        x.nb = sg.nb;
        x.ntiles = sg.ntiles;
        for (int32_t t = 0; t < sg.ntiles; ++t) tile_graph[tb + t] = i;
        for (int32_t b = 0; b < sg.nb; ++b) block_graph[bb + b] = i;
        voff += g.V;
        qoff += sg.Q;
        tb += sg.ntiles;
        bb += sg.nb;
    }
    CAGRA_HIP_CHECK(hipMemcpyAsync(m->desc, host.data(), m->desc_bytes, hipMemcpyHostToDevice, stream));
    CAGRA_HIP_CHECK(hipStreamSynchronize(stream));  // the host staging copy goes out of scope
    int dev = 0, cus = 0;
    CAGRA_HIP_CHECK(hipGetDevice(&dev));
    CAGRA_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    m->grid_gather = cus;      // one 160 KB-LDS workgroup per CU
    m->grid_merge = 2 * cus;
    return CAGRA_OK;
}

static cagra_status check_ready(const cagra_multi *m) {
    if (!m || m->ngraphs < 1 || !m->desc || m->grid_gather < 1 || m->grid_merge < 1)
        return fail(CAGRA_E_INVALID, "multi-graph plan is not set up");
    return CAGRA_OK;
}

cagra_status cagra_multi_pagerank_start(const cagra_multi *m, hipStream_t stream) {
    cagra_status s;
    if ((s = check_ready(m)) != CAGRA_OK) return s;
    const MultiDesc *d = reinterpret_cast<const MultiDesc *>(m->desc);
    const int32_t *block_graph =
        reinterpret_cast<const int32_t *>((const unsigned char *)m->desc + desc_area(m->ngraphs)) + m->total_tiles;
    return launch_multi_start(d, block_graph, m->total_blocks, m->ngraphs, m->blk, m->grid_merge, stream);
}

cagra_status cagra_multi_pagerank_step(const cagra_multi *m, int32_t parity, double damping, hipStream_t stream) {
    cagra_status s;
    if ((s = check_ready(m)) != CAGRA_OK) return s;
    if (parity != 0 && parity != 1) return fail(CAGRA_E_INVALID, "parity must be 0 or 1");
    if (!(damping >= 0.0 && damping <= 1.0)) return fail(CAGRA_E_INVALID, "damping must be in [0, 1]");
    const MultiDesc *d = reinterpret_cast<const MultiDesc *>(m->desc);
    const int32_t *tile_graph =
        reinterpret_cast<const int32_t *>((const unsigned char *)m->desc + desc_area(m->ngraphs));
    const int32_t *block_graph = tile_graph + m->total_tiles;
    if ((s = launch_multi_gather(d, tile_graph, m->total_tiles, parity, m->grid_gather, stream)) != CAGRA_OK)
        return s;
    return launch_multi_merge(d, block_graph, m->total_blocks, m->ngraphs, parity, damping, m->blk,
                              merge_fused_lds_bytes(m->max_B, m->max_k, 8), m->grid_merge, stream);
}

}  // extern "C"
