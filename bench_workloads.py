"""Secondary measurements for bench.py --workload (each prints one JSON line).

labelprop   min-label propagation, R-MAT scale 22 / ef 16 / seed 2, symmetrized,
            to the fixed point (GTEPS over the symmetric edge count)
ppr         personalized PageRank with 64 seed vertices at once (restart 0.15),
            R-MAT scale 22 / ef 16 / seed 4, 20 iterations; segment sizes from the
            autotuner's candidates; compared with the plain single-vector iteration
ppr         ...
multigraph  256 independent R-MAT graphs (scale U{10..20}, ef U{8..32}, seed 4),
            start + 20 iterations of all of them captured into one HIP graph,
            compared with running the graphs one after another
warmstart   MLP warm start trained on 200 R-MAT graphs (scale U{16..20}, ef 16,
            seeds 1000+i) from PageRank vectors the method computes; held-out
            R-MAT scale 24 / ef 24 / seed 5; iterations and time to L1 residual
            < 1e-6 from the learned start (features and network included) vs
            the uniform start
cf          collaborative filtering (gradient-descent matrix factorization, 64
            factors) on a Netflix-shaped synthetic rating graph: 2^19 users, 2^14
            items, R-MAT-drawn ratings (edge factor 200 per user, duplicates
            removed), each rating an edge in both directions; segment sizes swept
bc          betweenness centrality (Brandes) from 12 sampled starts on R-MAT scale
            25 / ef 32 / seed 3, level-synchronous segmented pulls with the frontier
            as a mask of active segments (forward on the graph, backward on its
            reverse)
push        push-direction segmenting (expand, per-piece LDS scatter, update):
            PageRank on R-MAT scale 25 / ef 32 / seed 3 through the segmentation
            of the reverse graph, segment sizes swept, against the pull iteration
            on the same graph; label propagation on the symmetrized R-MAT 22
            (push against pull, same segmentation)
nsweep      PageRank iteration time, Q and q per segment size N on R-MAT scale 25 /
            ef 32 / seed 3 (the headline graph): LDS-sized N (8,192 ... 40,960),
            an L2-sized N (2^20 vertices, 4 MB of FP32 values), an
            Infinity-Cache-sized N (2^24) and one segment (the plain pull)
cluster     frequency-based clustering (Section 5) then segmenting, R-MAT scale 25
            / ef 32 / seed 3 (the headline graph): clustering time, expansion
            factor q, PageRank iteration time and time to L1 residual < 1e-6,
            against segmenting alone on the same graph
"""
from __future__ import annotations

import time

import numpy as np


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(fn, reps, rounds=3):
    """ms per call: the median over `rounds` runs of `reps` back-to-back calls
    (one untimed call first), so that one disturbed run does not set it."""
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(rounds):
        a, b = _events()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) / reps)
    return float(np.median(out))


def labelprop(args, log):
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    g = graphgen.symmetrize(graphgen.rmat_graph(22, 16, 2))
    log(f"labelprop graph V={g.V} E_sym={g.E}")
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 32768, 8192, 262144)
    lab, it = cagra.labelprop(seg)  # warm-up and iteration count
    torch.cuda.synchronize()
    a, b = _events()
    a.record()
    lab, it = cagra.labelprop(seg)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    comps = int(torch.unique(lab).numel())
    return {"metric": "GTEPS per label-propagation iteration at R-MAT-22 (symmetrized)",
            "value": round(g.E * it / (ms * 1e-3) / 1e9, 3), "unit": "GTEPS", "iterations_to_fixed_point": it,
            "ms_total": round(ms, 3), "ms_per_iteration": round(ms / it, 4), "components": comps,
            "config": {"workload": "labelprop_rmat22_ef16_seed2_sym", "V": g.V, "E_sym": g.E, "N": 32768,
                       "B": 8192, "k": seg.k, "Q": seg.Q}, "dtype": "i32", "data": "synthetic"}


def ppr(args, log):
    """64-seed personalized PageRank on R-MAT 22 / ef 16 / seed 4 (restart 0.15):
    segment size, merge block and tile from the autotuner; per-iteration rate and
    time until every column's L1 residual is below 1e-6, against the plain
    single-vector form (one personalized iteration per seed, LDS-staged
    segments) run seed by seed to the same residual."""
    import torch
    import graphgen
    from paper_1608_01362_amd import autotune, cagra
    g = graphgen.rmat_graph(22, 16, 4)
    rng = np.random.default_rng(4)
    ok = np.where((np.diff(g.in_offsets) > 0) | (g.out_degree > 0))[0]
    seeds = rng.choice(ok, size=64, replace=False).astype(np.int32)
    dg = cagra.DeviceGraph.from_host(g)
    best, timed = autotune.tune_ppr(dg, seeds, cache_path=None, log=log)
    seg = cagra.build_segments(dg, best.N, best.B, best.tile_edges)
    st = cagra.PPRState(dg, seg, seeds)
    st.start()
    ms = _time(st.step, 20)
    # batched: until every column's residual is below 1e-6 (the library's solve
    # loop, once untimed first)
    st.solve(tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = st.solve(tol=1e-6)
    batched_ms = (time.perf_counter() - t0) * 1e3
    it_b, worst = rb.iters, rb.residual
    Rb = st.ranks().clone()
    # plain: the single-vector iteration per seed, LDS-staged segments
    seg1 = cagra.build_segments(dg, 32768, 8192, 65536)
    st1 = cagra.PageRankState(dg, seg1)
    st1.start()
    ms1 = _time(st1.step, 20)
    bufs = cagra.SolveBuffers(dg, seg1)
    cagra.pagerank_solve(dg, seg1, tol=1e-6, restart=int(seeds[0]), state=bufs)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, kept = [], {}
    for j, s in enumerate(seeds):
        r = cagra.pagerank_solve(dg, seg1, tol=1e-6, restart=int(s), state=bufs)
        its.append(r.iters)
        if j % 16 == 0:
            kept[j] = r.rank.clone()
    plain_ms = (time.perf_counter() - t0) * 1e3
    # the two forms agree (each within the contraction bound of the fixed point)
    l1 = max(float((kept[j].double() - Rb[:, j].double()).abs().sum().item()) for j in kept)
    out = {"metric": "edge-columns per second, 64-seed personalized PageRank at R-MAT-22",
           "value": round(g.E * 64 / (ms * 1e-3) / 1e9, 3), "unit": "G edge-columns/s",
           "ms_per_iteration": round(ms, 4), "plain_single_vector_ms_per_iteration": round(ms1, 4),
           "plain_single_vector_GTEPS": round(g.E / (ms1 * 1e-3) / 1e9, 3),
           "speedup_vs_64_plain_iterations": round(64 * ms1 / ms, 3),
           "time_to_l1_1e-6": {"batched": {"iterations": it_b, "ms": round(batched_ms, 3),
                                           "worst_column_residual": worst},
                               "plain_seed_by_seed": {"iterations_total": int(sum(its)), "ms": round(plain_ms, 3)},
                               "speedup": round(plain_ms / batched_ms, 3),
                               "max_l1_between_forms": l1},
           "config": {"workload": "ppr64_rmat22_ef16_seed4", "V": g.V, "E": g.E, "N": best.N, "B": best.B,
                      "tile_edges": best.tile_edges, "q": round(best.Q / g.V, 4), "columns": 64, "restart": 0.15},
           "autotune_trials": [{"N": c.N, "B": c.B, "tile_edges": c.tile_edges, "ms": round(c.ms, 4)}
                               for c in timed],
           "dtype": "f32", "data": "synthetic"}
    log(f"ppr64: {ms:.3f} ms/iteration; to 1e-6 batched {batched_ms:.1f} ms vs seed by seed {plain_ms:.1f} ms")
    return out


def multigraph(args, log):
    """256 uneven R-MAT graphs (scale U{10..20}, ef U{8..32}, seed 4): per size
    class N/B/T from the autotuner, start + 20 iterations of every graph in one
    captured launch, against the same iterations graph by graph."""
    import torch
    import graphgen
    from paper_1608_01362_amd import autotune, cagra
    specs = graphgen.multigraph_specs(256, seed=4)
    t0 = time.perf_counter()
    gs = [graphgen.rmat_graph(s.scale, s.edge_factor, s.seed) for s in specs]
    log(f"generated 256 graphs, E total {sum(g.E for g in gs)} in {time.perf_counter() - t0:.1f}s")
    dgs = [cagra.DeviceGraph.from_host(g) for g in gs]
    Etot = sum(g.E for g in gs)
    Vtot = int(sum(g.V for g in gs))
    del gs
    choice, trials = autotune.tune_multi(dgs, cache_path=None, log=log)
    segs = autotune.multi_segments(dgs, choice)
    mp = cagra.MultiPageRank(dgs, segs)
    mp.capture(20)
    torch.cuda.synchronize()
    a, b = _events()
    reps = 3
    a.record()
    for _ in range(reps):
        mp.replay()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    res20 = mp.scalars[mp.cur].view(-1, 4)[:, 1].max().item()
    # the same work graph by graph, eager launches, the default single-graph layout
    segs1 = [cagra.build_segments(d, min(32768, d.V), 8192, 65536) for d in dgs]
    states = [cagra.PageRankState(d, s) for d, s in zip(dgs, segs1)]
    torch.cuda.synchronize()
    a.record()
    for st in states:
        st.start()
        for _ in range(20):
            st.step()
    b.record()
    torch.cuda.synchronize()
    ms_seq = a.elapsed_time(b)
    out = {"metric": "aggregate GTEPS, 256 uneven R-MAT graphs x 20 PageRank iterations in one captured launch",
           "value": round(Etot * 20 / (ms * 1e-3) / 1e9, 3), "unit": "GTEPS", "ms_total": round(ms, 3),
           "graph_by_graph_ms": round(ms_seq, 3), "speedup_vs_graph_by_graph": round(ms_seq / ms, 3),
           "max_residual_after_20": res20,
           "tuned_per_size_class": {str(c): list(v) for c, v in choice.items()},
           "autotune_trials": len(trials),
           "config": {"workload": "multigraph256_rmat_s10-20_ef8-32_seed4", "graphs": 256, "E_total": Etot,
                      "V_total": Vtot, "tiles": int(mp.m.total_tiles), "blocks": int(mp.m.total_blocks)},
           "dtype": "f32", "data": "synthetic"}
    log(f"multigraph: {ms:.2f} ms for 20 iterations of 256 graphs vs {ms_seq:.1f} ms graph by graph")
    return out


def warmstart(args, log, oracle_star=True):
    """Learned warm start: network trained on 200 R-MAT graphs (scale U{16..20},
    ef 16) from the method's own PageRank vectors, held-out R-MAT 24 / ef 24 /
    seed 5; time to L1 residual < 1e-6 from the learned start (features,
    network and softmax included) against the uniform start."""
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    from paper_1608_01362_amd import warmstart as ws
    t0 = time.perf_counter()
    Fs, Ts, rows = [], [], 0
    for sp in graphgen.warmstart_training_specs():
        g = graphgen.rmat_graph(sp.scale, sp.edge_factor, sp.seed)
        dg = cagra.DeviceGraph.from_host(g)
        seg = cagra.build_segments(dg, 32768, 8192, 65536)
        Fs.append(ws.features(dg, seg))
        Ts.append(ws.pagerank_target(dg, seg))
        rows += g.V
        del dg, seg
    F, T = torch.cat(Fs), torch.cat(Ts)
    del Fs, Ts
    log(f"training data: {rows} rows from 200 graphs in {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = ws.train(F, T, seed=0, steps=600, batch=65536, lr=3e-3, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del F, T
    gt = graphgen.rmat_graph(24, 24, 5)
    dg = cagra.DeviceGraph.from_host(gt)
    seg = cagra.build_segments(dg, 32768, 8192, 262144)
    import ctypes
    wsp = torch.empty(cagra.lib().cagra_learned_start_workspace_bytes(ctypes.byref(seg.c)), dtype=torch.uint8,
                      device="cuda")
    bufs = cagra.SolveBuffers(dg, seg)
    ws.solve(dg, seg, tol=1e-6, buffers=bufs)  # warm-up of both paths
    ws.solve(dg, seg, tol=1e-6, net=net, ws=wsp, buffers=bufs)
    runs_u, runs_w = [], []
    for _ in range(5):  # interleaved, so that clock drift affects both alike
        r = ws.solve(dg, seg, tol=1e-6, buffers=bufs)
        runs_u.append((r[0].clone(), *r[1:]))
        r = ws.solve(dg, seg, tol=1e-6, net=net, ws=wsp, buffers=bufs)
        runs_w.append((r[0].clone(), *r[1:]))
    r_u, it_u, _, _ = runs_u[0]
    r_w, it_w, _, used = runs_w[0]
    ms_u = float(np.median([r[2] for r in runs_u]))
    ms_w = float(np.median([r[2] for r in runs_w]))
    # the start vector's own cost, and its parts
    start_ms = _time(lambda: ws.learned_start(net, dg, seg, wsp), 5)
    F = ws.features(dg, seg)
    feat_ms = _time(lambda: ws.features(dg, seg), 5)
    y = net.forward(F)
    fwd_all_ms = _time(lambda: net.forward(F), 5)
    unfused_ms = _time(lambda: ws.start_vector(net, ws.features(dg, seg)), 5)
    del F, y
    l1 = float((r_u.double() - r_w.double()).abs().sum().item())
    out = {"metric": "time to L1 residual < 1e-6, learned warm start vs uniform, held-out R-MAT-24",
           "value": round(ms_w, 3), "unit": "ms", "higher_is_better": False,
           "uniform": {"iterations": it_u, "ms": round(ms_u, 3)},
           "learned": {"iterations": it_w, "ms": round(ms_w, 3), "start_used": used,
                       "start_vector_ms": round(start_ms, 3),
                       "parts_ms": {"features": round(feat_ms, 3), "network_every_row": round(fwd_all_ms, 3),
                                    "unfused_start": round(unfused_ms, 3)}},
           "speedup": round(ms_u / ms_w, 3), "l1_between_answers": l1,
           "training": {"graphs": 200, "rows": rows, "steps": 600, "batch": 65536, "seconds": round(train_s, 2),
                        "loss_first": net.losses[0], "loss_last": net.losses[-1]},
           "config": {"workload": "warmstart_rmat24_ef24_seed5", "V": gt.V, "E": gt.E, "N": 32768, "B": 8192},
           "dtype": "f32 iteration, bf16-weight network", "data": "synthetic"}
    if oracle_star:
        import oracle
        star, _ = oracle.pagerank(gt, iters=300, tol=1e-11, threads=min(16, len(__import__("os").sched_getaffinity(0))))
        out["uniform"]["l1_to_oracle_fixed_point"] = float(np.abs(r_u.double().cpu().numpy() - star).sum())
        out["learned"]["l1_to_oracle_fixed_point"] = float(np.abs(r_w.double().cpu().numpy() - star).sum())
    log(f"warmstart: uniform {it_u} it {ms_u:.2f} ms, learned {it_w} it {ms_w:.2f} ms (start {start_ms:.2f} ms)")
    return out


def _pagerank_timing(cagra, dg, seg, steps, warmup):
    import torch
    st = cagra.PageRankState(dg, seg)
    st.start()
    for _ in range(warmup):
        st.step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for i in range(steps):
        st.step_split(events=evs[i])
    torch.cuda.synchronize()
    g_ms = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    m_ms = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    total = evs[0][0].elapsed_time(evs[-1][2]) / steps
    return total, g_ms, m_ms


def cluster(args, log):
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    g = graphgen.rmat_graph(25, 32, 3)
    log(f"graph V={g.V} E={g.E}")
    dg = cagra.DeviceGraph.from_host(g)
    del g
    N, B, T = 32768, 8192, 262144
    res = {}
    cagra.cluster(dg)  # warm-up (first use of the sort kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cg, perm, H = cagra.cluster(dg)
    torch.cuda.synchronize()
    cl_ms = (time.perf_counter() - t0) * 1e3
    log(f"clustered: H={H} ({100.0 * H / dg.V:.1f}% of vertices) in {cl_ms:.1f} ms")
    for name, gg in (("segmenting", dg), ("clustering+segmenting", cg)):
        t0 = time.perf_counter()
        seg = cagra.build_segments(gg, N, B, T)
        torch.cuda.synchronize()
        b_ms = (time.perf_counter() - t0) * 1e3
        total, g_ms, m_ms = _pagerank_timing(cagra, gg, seg, 20, 3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, resid, it = cagra.pagerank(gg, seg, iters=100, tol=1e-6)
        conv_ms = (time.perf_counter() - t1) * 1e3
        res[name] = {"q": round(seg.q, 4), "Q": seg.Q, "build_ms": round(b_ms, 2), "ms_per_iter": round(total, 4),
                     "gather_ms": round(g_ms, 4), "merge_ms": round(m_ms, 4),
                     "gteps": round(dg.E / (total * 1e-3) / 1e9, 2),
                     "to_l1_1e-6": {"iterations": it, "ms": round(conv_ms, 2), "final_residual": resid[-1]}}
        log(f"{name}: {res[name]}")
        del seg
    c, p = res["clustering+segmenting"], res["segmenting"]
    return {"metric": "GTEPS per PageRank iter at R-MAT-25 after frequency-based clustering",
            "value": c["gteps"], "unit": "GTEPS", "higher_is_better": True,
            "vs_segmenting_alone": round(c["gteps"] / p["gteps"], 3),
            "clustering_ms": round(cl_ms, 2), "clustered_vertices": H, **res,
            "config": {"workload": "pagerank_rmat25_ef32_seed3_clustered", "V": dg.V, "E": dg.E,
                       "N": N, "B": B, "tile_edges": T},
            "dtype": "f32", "data": "synthetic"}


def cf(args, log):
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    t0 = time.perf_counter()
    g, vals, U, I = graphgen.bipartite_ratings(19, 14, 200, 6)
    log(f"rating graph: {U} users, {I} items, {g.E // 2} ratings ({g.E} in-edges) in {time.perf_counter() - t0:.1f}s")
    dg = cagra.DeviceGraph.from_host(g)
    vals_d = torch.from_numpy(vals).cuda()
    rng = np.random.default_rng(9)
    x0 = torch.from_numpy((rng.random((g.V, cagra.CF_FACTORS)) * 0.1).astype(np.float32)).cuda()
    E = g.E
    del g, vals
    gamma, lam, steps = 3e-5, 0.05, 10  # below 2 / (largest Hessian eigenvalue) for the heaviest items
    trials = []
    for N in (8192, 16384, 65536, 262144, dg.V):
        seg = cagra.build_segments(dg, N, 512)
        sv = cagra.segment_edge_values(dg, seg, vals_d)
        st = cagra.CFState(dg, seg, sv, x0)
        st.step(gamma, lam)
        st.step(gamma, lam)
        ms = _time(lambda: st.step(gamma, lam), steps)
        trials.append({"N": N, "k": seg.k, "q": round(seg.q, 4), "ms_per_step": round(ms, 4)})
        log(f"cf N={N} k={seg.k} q={seg.q:.3f}: {ms:.3f} ms per step")
        del st, sv, seg
        torch.cuda.empty_cache()
    best = min(trials, key=lambda t: t["ms_per_step"])
    seg = cagra.build_segments(dg, best["N"], 512)
    st = cagra.CFState(dg, seg, cagra.segment_edge_values(dg, seg, vals_d), x0)
    rmse = []
    for _ in range(steps):
        st.step(gamma, lam)
        rmse.append(round(float(np.sqrt(st.sq.item() / E)), 5))
    one = [t for t in trials if t["k"] == 1][0]
    ms = best["ms_per_step"]
    return {"metric": "GTEPS per collaborative-filtering step (64 factors) on a Netflix-shaped rating graph",
            "value": round(E / (ms * 1e-3) / 1e9, 3), "unit": "GTEPS", "ms_per_step": ms,
            "edge_factor_updates_per_s_G": round(E * cagra.CF_FACTORS / (ms * 1e-3) / 1e9, 1),
            "best_segment_vertices": best["N"], "one_segment_ms_per_step": one["ms_per_step"],
            "speedup_vs_one_segment": round(one["ms_per_step"] / ms, 3), "trials": trials,
            "rmse_per_step": rmse, "gamma": gamma, "lambda": lam,
            "config": {"workload": "cf_ratings_u19_i14_ef200_seed6", "users": U, "items": I, "in_edges": E,
                       "factors": cagra.CF_FACTORS, "B": 512},
            "dtype": "f32", "data": "synthetic"}


def bc(args, log):
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    t0 = time.perf_counter()
    g = graphgen.rmat_graph(25, 32, 3)
    gt = graphgen.transpose(g)
    log(f"graph and reverse in {time.perf_counter() - t0:.1f}s")
    rng = np.random.default_rng(12)
    sources = rng.choice(np.flatnonzero(g.out_degree > 0), size=12, replace=False)
    dg, dgt = cagra.DeviceGraph.from_host(g), cagra.DeviceGraph.from_host(gt)
    V, E = g.V, g.E
    del g, gt
    seg = cagra.build_segments(dg, 32768, 8192, 262144)
    seg_t = cagra.build_segments(dgt, 32768, 8192, 262144)
    st = cagra.BCState(seg, seg_t)
    st.add_source(int(sources[0]))  # warm-up
    st.bc.zero_()
    st.levels = []
    torch.cuda.synchronize()
    per = []
    t1 = time.perf_counter()
    for s_ in sources:
        a = time.perf_counter()
        st.add_source(int(s_))
        torch.cuda.synchronize()
        per.append(round((time.perf_counter() - a) * 1e3, 2))
    total = time.perf_counter() - t1
    log(f"12 starts: {total * 1e3:.1f} ms; per start {per}; BFS levels {st.levels}")
    passes = sum(2 * lv - 1 for lv in st.levels)  # forward levels + backward levels
    return {"metric": "seconds for betweenness centrality from 12 starts at R-MAT-25", "value": round(total, 4),
            "unit": "s", "higher_is_better": False, "ms_per_start": per, "bfs_levels": st.levels,
            "segmented_passes": passes, "dense_equivalent_GTEPS": round(E * passes / total / 1e9, 2),
            "config": {"workload": "bc12_rmat25_ef32_seed3", "V": V, "E": E, "N": 32768, "B": 8192,
                       "sources": [int(x) for x in sources]},
            "dtype": "f32", "data": "synthetic"}


def push(args, log):
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    t0 = time.perf_counter()
    g = graphgen.rmat_graph(25, 32, 3)
    gt = graphgen.transpose(g)
    log(f"graph and reverse in {time.perf_counter() - t0:.1f}s")
    dg, dgt = cagra.DeviceGraph.from_host(g), cagra.DeviceGraph.from_host(gt)
    V, E = g.V, g.E
    del g, gt
    steps = max(args.steps, 5)
    sweep = {}
    best = None
    for N in ((args.push_n,) if args.push_n else (8192, 16384, 20480)):
        seg_t = cagra.build_segments(dgt, N, 8192, 262144)
        st = cagra.PushPageRankState(dg, seg_t)
        st.start()
        ms = _time(st.step, steps)
        sweep[N] = {"ms_per_iter": round(ms, 4), "GTEPS": round(E / ms / 1e6, 1), "k": seg_t.k,
                    "q": round(seg_t.q, 3)}
        log(f"push N={N}: {ms:.3f} ms/iter, q={seg_t.q:.3f}")
        if best is None or ms < sweep[best]["ms_per_iter"]:
            best = N
        del st, seg_t
        torch.cuda.empty_cache()
    it, conv_ms = None, None
    if not args.no_converge:
        seg_t = cagra.build_segments(dgt, best, 8192, 262144)
        r, res, it = cagra.pagerank_push(dg, seg_t, iters=100, tol=1e-6)
        torch.cuda.synchronize()
        a, b = _events()
        a.record()
        cagra.pagerank_push(dg, seg_t, iters=it)
        b.record()
        torch.cuda.synchronize()
        conv_ms = round(a.elapsed_time(b), 2)
        del seg_t
    seg = cagra.build_segments(dg, 32768, 8192, 262144)
    stp = cagra.PageRankState(dg, seg)
    stp.start()
    pull_ms = _time(stp.step, steps)
    log(f"pull N=32768: {pull_ms:.3f} ms/iter; push best N={best}: {sweep[best]['ms_per_iter']:.3f}")
    del stp, seg, dg, dgt
    torch.cuda.empty_cache()
    # label propagation on the symmetrized R-MAT 22: push and pull on one segmentation
    gs = graphgen.symmetrize(graphgen.rmat_graph(22, 16, 2))
    dgs = cagra.DeviceGraph.from_host(gs)
    segs = cagra.build_segments(dgs, 32768, 8192, 262144)
    lab_push, it_push = cagra.labelprop_push(segs)
    torch.cuda.synchronize()
    a, b = _events()
    a.record()
    cagra.labelprop_push(segs)
    b.record()
    torch.cuda.synchronize()
    lp_push_ms = a.elapsed_time(b)
    a.record()
    lab_pull, it_pull = cagra.labelprop(segs)
    b.record()
    torch.cuda.synchronize()
    lp_pull_ms = a.elapsed_time(b)
    assert torch.equal(lab_push, lab_pull) and it_push == it_pull
    pm = sweep[best]["ms_per_iter"]
    return {"metric": "GTEPS per push-direction PageRank iteration at R-MAT-25", "value": round(E / pm / 1e6, 1),
            "unit": "GTEPS", "higher_is_better": True, "ms_per_iter": pm, "best_N": best, "sweep": sweep,
            "pull_ms_per_iter": round(pull_ms, 4), "push_over_pull_time": round(pm / pull_ms, 3),
            "iters_to_1e-6": it, "ms_to_1e-6": conv_ms,
            "labelprop_rmat22_sym": {"E_sym": gs.E, "iterations": it_push, "push_ms": round(lp_push_ms, 2),
                                     "pull_ms": round(lp_pull_ms, 2),
                                     "push_GTEPS": round(gs.E * it_push / lp_push_ms / 1e6, 1),
                                     "pull_GTEPS": round(gs.E * it_pull / lp_pull_ms / 1e6, 1)},
            "config": {"workload": "pagerank_push_rmat25_ef32_seed3", "V": V, "E": E, "B": 8192,
                       "tile_edges": 262144},
            "dtype": "f32", "data": "synthetic"}


def nsweep(args, log):
    import torch
    import graphgen
    from paper_1608_01362_amd import cagra
    g = graphgen.rmat_graph(args.scale, args.edge_factor, args.seed)
    dg = cagra.DeviceGraph.from_host(g)
    rows = []
    for N in (8192, 16384, 24576, 32768, 40960, 1 << 20, 1 << 24, g.V):
        seg = cagra.build_segments(dg, N, args.B, args.tile_edges)
        total, g_ms, m_ms = _pagerank_timing(cagra, dg, seg, 10, 2)
        rows.append({"N": N, "k": seg.k, "Q": seg.Q, "q": round(seg.q, 3),
                     "edge_word_bytes": 2 if N <= cagra.EDGE16_MAX_N else 4,
                     "ms_per_iteration": round(total, 4), "gather_ms": round(g_ms, 4), "merge_ms": round(m_ms, 4),
                     "GTEPS": round(g.E / (total * 1e-3) / 1e9, 2)})
        log(f"N={N}: k={seg.k} q={seg.q:.3f} {total:.3f} ms/iter (gather {g_ms:.3f}, merge {m_ms:.3f})")
        del seg
        torch.cuda.empty_cache()
    return {"metric": "PageRank ms per iteration by segment size", "unit": "ms", "data": "synthetic",
            "config": {"workload": f"pagerank_rmat{args.scale}_ef{args.edge_factor}_seed{args.seed}",
                       "V": g.V, "E": g.E, "B": args.B, "tile_edges": args.tile_edges}, "rows": rows}


def run(name, args, log):
    return {"labelprop": labelprop, "ppr": ppr, "multigraph": multigraph, "warmstart": warmstart,
            "cluster": cluster, "cf": cf, "bc": bc, "push": push, "nsweep": nsweep}[name](args, log)
