"""Benchmark: exact prime paths + test paths of one ~200-vertex structured CFG
on one MI355X.

One step = one pass of the whole hot path on the GPU: level-synchronous
extension of simple paths from every vertex, backward-extendability filter,
canonical ordering and materialization of the prime paths, BFS tables, splice
of every prime path into a test path, sort and deduplication.  The input CSR
is resident in HBM before timing starts and results stay in HBM.

Prints one JSON line (see the fields below).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "prime paths/s + path-extensions/s, exact; batched+learned vs plain on 1 GPU"


def _workload():
    from paper_2210_16998_amd import cfggen
    with open(os.path.join(ROOT, "tests", "golden", "workloads.json")) as f:
        w = json.load(f)
    rec = max(w["c2"], key=lambda r: r["n_pp"])
    return cfggen.c2_cfg(rec["seed"]), rec


def _kernel_name(W: int, tuning, g) -> str:
    """Name of the extension-kernel instantiation the library runs for
    visited sets of W words under this tuning on graph g (mirrors the
    dispatch: the thread-per-parent kernel stages the CSR in LDS when its
    3n + 2m + 4 words fit in 16 KiB)."""
    i = W.bit_length() - 1
    items, var = tuning["items"][i], tuning["variant"][i]
    if var != 0:
        while items > 1 and items * W > 32:
            items //= 2
    if var != 0 and items * W <= 32:
        staged = "true" if 4 * (3 * g.n + 2 * g.n_edges + 4) <= 16384 else "false"
        return f"k_extend_tp<{W}, {items}, {256 if var == 1 else 1024}, {staged}>"
    return f"k_extend_lb<{W}, {items}>"


def _copy_peak(stream, mib: int = 4096, reps: int = 10) -> float:
    """Achievable HBM bandwidth of a plain device-to-device copy (GB/s,
    bytes read + written), the second denominator beside the published peak."""
    import torch
    with torch.cuda.stream(stream):
        src = torch.ones(mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        best = float("inf")
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dst.copy_(src)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def _measured_traffic(kernel: str, summary: str = "k_extend_cfg209_hbm_traffic.md"):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on this same kernel (else None)."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        for line in open(path):
            line = line.strip()
            if line.startswith("traffic kernel="):
                name = line[len("traffic kernel="):line.index(" bytes_per_launch=")]
                val = float(line.split("bytes_per_launch=")[1].split()[0])
                return val if name == kernel else None
    except OSError:
        return None
    return None


def _bytes_per_extension(n: int) -> int:
    """Algorithmic HBM bytes per path extension: the child's 8-byte record is
    written once and read once as a parent (16 B), and its visited set of
    ceil(n / 64) words is written once and read once."""
    return 16 + 2 * 8 * ((n + 63) // 64)


def _stress(args, copy_gbs: float):
    """The 400-vertex stress CFG: one-pass prime paths (device output), with
    the extension kernel's roofline measured on its ~4.7e8 extensions."""
    import torch
    from paper_2210_16998_amd import cfggen, tpg
    g = cfggen.c5_cfg()
    h = tpg.load_cfg(g)
    ws = tpg.Workspace(0)
    stream = torch.cuda.Stream()
    cap = 64 << 30  # the stress workload's pool cap (64 GiB of HBM)
    tpg.prime_paths(h, ws=ws, flags=tpg.TPG_OUT_DEVICE, stream=stream, pool_cap=cap)
    torch.cuda.synchronize()
    times, k_ms, k_launches = [], 0.0, 0
    for _ in range(args.stress_reps):
        t = time.perf_counter()
        _, st = tpg.prime_paths(h, ws=ws, flags=tpg.TPG_OUT_DEVICE, stream=stream, pool_cap=cap)
        times.append(time.perf_counter() - t)
        k_ms += st["ms_extend_kernel"]
        k_launches += st["n_extend_launches"]
    bpe = _bytes_per_extension(g.n)
    avg = k_ms / max(1, k_launches)
    per_launch = st["n_extensions"] * bpe / max(1, st["n_extend_launches"])
    ach = per_launch / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
    ms = 1000.0 * statistics.median(times)
    kname = _kernel_name(8, tpg.get_tuning(ws), g)
    traffic = _measured_traffic(kname, "k_extend_stress400_hbm_traffic.md")
    ws.close()
    return {"workload": f"stress CFG, {g.n} vertices, {g.n_edges} arcs (3 nested whiles, 16-way "
                        f"switch, 60 diamonds), prime paths only",
            "n_pp": st["n_pp"], "n_extensions": st["n_extensions"], "levels": st["n_levels"],
            "ms_per_run_median": ms, "prime_paths_per_s": st["n_pp"] / (ms * 1e-3),
            "extensions_per_s": st["n_extensions"] / (ms * 1e-3),
            "extend_kernel_ms": k_ms / args.stress_reps,
            "device_bytes": st["device_bytes"], "pool_cap_bytes": cap,
            "roofline": {"bound": "hbm", "kernel": kname, "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                         "traffic": traffic,
                         "measured_GBps": traffic / (avg * 1e-3) / 1e9 if traffic and avg > 0 else None,
                         "copy_GBps": copy_gbs, "frac_of_copy": ach / copy_gbs,
                         "algorithmic_bytes_per_launch": per_launch,
                         "bytes_per_extension": bpe, "launches_per_run": st["n_extend_launches"],
                         "avg_launch_ms": avg}}


def _paper_form(args):
    """The same CFG in the paper's input form (switch vertices binarized to
    out-degree 2 at load): whole path per step, and the prime paths grouped by
    last vertex (the paper's per-end-vertex output) against canonical order."""
    import torch
    from paper_2210_16998_amd import tpg
    g, rec = _workload()
    h = tpg.load_cfg(g, tpg.TPG_LOAD_BINARIZE)
    n_b, m_b, _, _ = h.info()
    ws = tpg.Workspace(0)
    stream = torch.cuda.Stream()
    f = tpg.TPG_OUT_DEVICE | tpg.TPG_NO_TIMING

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - t) / reps

    ms = timed(lambda: tpg.test_paths(h, ws=ws, flags=f, stream=stream), args.steps)
    _, _, st = tpg.test_paths(h, ws=ws, flags=tpg.TPG_OUT_DEVICE, stream=stream)
    h0 = tpg.load_cfg(g)
    ms_pp = timed(lambda: tpg.prime_paths(h0, ws=ws, flags=f, stream=stream), args.steps)
    ms_last = timed(lambda: tpg.prime_paths(h0, ws=ws, flags=f | tpg.TPG_ORDER_BY_LAST,
                                            stream=stream), args.steps)
    ws.close()
    return {"workload": f"the benchmark CFG binarized: {n_b} vertices, {m_b} arcs (from {g.n}, "
                        f"{g.n_edges})",
            "n_pp": st["n_pp"], "n_extensions": st["n_extensions"], "n_tp": st["n_tp"],
            "ms_per_step": ms, "prime_paths_per_s": st["n_pp"] / (ms * 1e-3),
            "grouped_by_last": {"prime_paths_ms": ms_pp, "grouped_ms": ms_last,
                                "overhead_ms": ms_last - ms_pp}}


def _covering(args):
    """Test paths by longest-first covering (TPG_TP_GREEDY) on the benchmark
    CFG: whole path per step, against the plain splice + dedup."""
    import torch
    from paper_2210_16998_amd import tpg
    g, rec = _workload()
    h = tpg.load_cfg(g)
    ws = tpg.Workspace(0)
    stream = torch.cuda.Stream()
    out = {}
    for name, fl in (("plain", 0), ("greedy", tpg.TPG_TP_GREEDY)):
        f = tpg.TPG_OUT_DEVICE | fl
        for _ in range(2):
            tpg.test_paths(h, ws=ws, flags=f | tpg.TPG_NO_TIMING, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            tpg.test_paths(h, ws=ws, flags=f | tpg.TPG_NO_TIMING, stream=stream)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t) / args.steps
        _, _, st = tpg.test_paths(h, ws=ws, flags=f, stream=stream)
        out[name] = {"ms_per_step": ms, "n_tp": st["n_tp"], "ms_tp": st["ms_tp"]}
    ws.close()
    out["workload"] = (f"the benchmark CFG ({g.n} vertices): test paths of the longest-first "
                       f"covering vs splice + dedup, whole path per step")
    return out


def _components(args):
    """Strongly connected components and prime-path types (Sec. 2) on the
    benchmark CFG: the device SCC pass, and the classification of its
    device-resident prime-path set (counts only)."""
    import torch
    from paper_2210_16998_amd import tpg
    g, rec = _workload()
    h = tpg.load_cfg(g)
    ws = tpg.Workspace(0)
    stream = torch.cuda.Stream()
    pp, _ = tpg.prime_paths(h, ws=ws, flags=tpg.TPG_OUT_DEVICE | tpg.TPG_NO_TIMING, stream=stream)
    out = {}
    for name, fn in (("scc_ms", lambda: tpg.scc(h, ws=ws, stream=stream)),
                     ("types_ms", lambda: tpg.prime_path_types(h, pp, ws=ws, stream=stream,
                                                               want_types=False))):
        for _ in range(3):
            r = fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
        torch.cuda.synchronize()
        out[name] = 1000.0 * (time.perf_counter() - t) / args.steps
        if name == "scc_ms":
            comp, fl = r[0], r[1]
            out["n_components"] = r[2]
            out["n_components_with_cycle"] = int(len(set(comp[(fl & tpg.TPG_SCC_CYCLIC) > 0].tolist())))
        else:
            names = ["", "complete", "scc_internal", "scc_exit", "scc_entry", "other"]
            out["types"] = {names[t]: int(r[1][t]) for t in range(1, 6)}
    ws.close()
    out["workload"] = (f"the benchmark CFG ({g.n} vertices, {out['n_components']} components): "
                       f"device SCC pass, and the types of its {len(pp)} prime paths held on the "
                       f"device (each call includes the graph upload and the SCC pass)")
    return out


def _prior_schedule(args):
    """The paper's per-vertex schedule (comparison variant) against the path
    tree, both giving the prime paths grouped by end vertex.  Its lists copy
    whole paths and one thread serves each vertex, so it is run on a while
    loop around 12 if-else diamonds (163 841 prime paths), not on the
    benchmark CFG."""
    import torch
    from paper_2210_16998_amd import cfggen, tpg
    k = 12
    g = cfggen.loop_diamond_chain(k)
    h = tpg.load_cfg(g)
    ws = tpg.Workspace(0)
    stream = torch.cuda.Stream()
    out = {}
    for name, fn in (("vertex_lists", tpg.prime_paths_vertex_lists),
                     ("path_tree", lambda h, **kw: tpg.prime_paths(
                         h, **{**kw, "flags": kw["flags"] | tpg.TPG_ORDER_BY_LAST}))):
        f = tpg.TPG_OUT_DEVICE | tpg.TPG_NO_TIMING
        fn(h, ws=ws, flags=f, stream=stream)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        t = time.perf_counter()
        for _ in range(reps):
            _, st = fn(h, ws=ws, flags=f, stream=stream)
        torch.cuda.synchronize()
        out[name] = {"ms_per_call": 1000.0 * (time.perf_counter() - t) / reps,
                     "n_pp": st["n_pp"], "n_extensions": st["n_extensions"]}
    ws.close()
    out["slowdown"] = out["vertex_lists"]["ms_per_call"] / out["path_tree"]["ms_per_call"]
    out["workload"] = (f"while loop around {k} if-else diamonds ({g.n} vertices, "
                       f"{(3 * k + 4) * 2 ** k + 1} prime paths), prime paths grouped by end vertex")
    return out


def _cpu_baseline(g, reps: int):
    """The CPU oracle on the same graph (DFS enumeration from every vertex,
    local-rule prime test, splice + sort + dedup of test paths)."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    n_pp = 0
    for _ in range(reps):
        pp, st = oracle.prime_paths_local(g, 0, g.n, nthreads=threads)
        tp, _ = oracle.test_paths(g, pp)
        n_pp += len(pp)
    dt = time.perf_counter() - t0
    # one core, on the start vertices 0 .. n/8 (a bounded sample)
    hi = max(1, g.n // 8)
    t1 = time.perf_counter()
    pp1, _ = oracle.prime_paths_local(g, 0, hi, nthreads=1)
    oracle.test_paths(g, pp1)
    dt1 = time.perf_counter() - t1
    return {"value": n_pp / dt, "unit": "prime paths/s", "cores": threads, "kind": "oracle",
            "sample": f"whole workload x{reps}: DFS from all {g.n} vertices with the local "
                      f"prime test, then test-path splice/sort/dedup; {dt:.1f} s total",
            "one_core": {"value": len(pp1) / dt1, "unit": "prime paths/s", "cores": 1,
                         "sample": f"start vertices 0..{hi - 1} ({len(pp1)} prime paths), same "
                                   f"steps; {dt1:.1f} s"}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--stress-reps", type=int, default=3)
    ap.add_argument("--no-paper-form", action="store_true")
    ap.add_argument("--no-covering", action="store_true")
    ap.add_argument("--no-components", action="store_true")
    ap.add_argument("--no-prior-schedule", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path is "
              f"single-GPU in this build", file=sys.stderr)
        return 2

    import torch
    from paper_2210_16998_amd import tpg

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    g, rec = _workload()
    ws = tpg.Workspace(0)
    h = tpg.load_cfg(g)
    stream = torch.cuda.Stream()
    flags = tpg.TPG_OUT_DEVICE

    def step(f=flags):
        return tpg.test_paths(h, ws=ws, flags=f, stream=stream, want_pp=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: every call returns after its stream has drained; the
    # level loop is replayed from captured HIP graphs
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        step(flags | tpg.TPG_NO_TIMING)
        times.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1000.0 * dt / args.steps
    # kernel-timed pass over the same steps: the same launches issued one by
    # one with a HIP event pair on the library's stream around every
    # extension launch, plus per-phase events
    k_ms, k_launches, phases = 0.0, 0, []
    t2 = time.perf_counter()
    for _ in range(args.steps):
        pp, tp, st = step()
        k_ms += st["ms_extend_kernel"]
        k_launches += st["n_extend_launches"]
        phases.append(st)
    torch.cuda.synchronize()
    ms_timed = 1000.0 * (time.perf_counter() - t2) / args.steps
    n_pp, n_ext = st["n_pp"], st["n_extensions"]
    bytes_per_ext = _bytes_per_extension(g.n)
    avg_launch_ms = k_ms / max(1, k_launches)
    # algorithmic bytes of one launch: the run's extensions spread over its launches
    achieved = (n_ext * bytes_per_ext / max(1, st["n_extend_launches"])) / (avg_launch_ms * 1e-3) / 1e9 \
        if avg_launch_ms > 0 else 0.0

    # plain per-CFG two-pass form, same graph, for context
    for _ in range(2):
        step(flags | tpg.TPG_FORCE_TWO_PASS | tpg.TPG_NO_TIMING)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    reps2 = max(3, args.steps // 4)
    for _ in range(reps2):
        step(flags | tpg.TPG_FORCE_TWO_PASS | tpg.TPG_NO_TIMING)
    torch.cuda.synchronize()
    ms_plain = 1000.0 * (time.perf_counter() - t1) / reps2

    def med(key):
        return statistics.median(p[key] for p in phases)

    W = 1
    while W * 64 < g.n:
        W *= 2
    kname = _kernel_name(W, tpg.get_tuning(ws), g)
    traffic = _measured_traffic(kname)
    copy_gbs = _copy_peak(stream)

    out = {
        "metric": METRIC,
        "value": n_pp / (ms * 1e-3),
        "unit": "prime paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"single structured CFG, {g.n} vertices, {g.n_edges} arcs, "
                               f"cyclomatic {g.cyclomatic}, seed {rec['seed']} (prime + test paths)",
                   "n_pp": n_pp, "n_extensions": n_ext, "n_tp": st["n_tp"],
                   "levels": st["n_levels"]},
        "extensions_per_s": n_ext / (ms * 1e-3),
        "test_paths_per_s": st["n_tp"] / (ms * 1e-3),
        "step_ms": {"median": 1000.0 * statistics.median(times),
                    "mean": 1000.0 * statistics.fmean(times),
                    "kernel_timed_pass_mean": ms_timed},
        "phase_ms_median": {"extend": med("ms_extend"), "rank_materialize": med("ms_rank"),
                            "test_paths": med("ms_tp"), "total_device": med("ms_total"),
                            "extend_kernel": med("ms_extend_kernel")},
        "plain_two_pass_ms_per_step": ms_plain,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "measured_GBps": traffic / (avg_launch_ms * 1e-3) / 1e9
                     if traffic and avg_launch_ms > 0 else None,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "algorithmic_bytes_per_launch": n_ext * bytes_per_ext / max(1, st["n_extend_launches"]),
                     "bytes_per_extension": bytes_per_ext,
                     "launches_per_step": st["n_extend_launches"],
                     "avg_launch_ms": avg_launch_ms},
    }
    if not args.no_stress:
        out["stress"] = _stress(args, copy_gbs)
    if not args.no_paper_form:
        out["paper_form"] = _paper_form(args)
    if not args.no_covering:
        out["covering"] = _covering(args)
    if not args.no_components:
        out["components"] = _components(args)
    if not args.no_prior_schedule:
        out["prior_schedule"] = _prior_schedule(args)
    if not args.no_batch:
        out["batched"] = _batched(args)
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(g, args.cpu_reps)
    print(json.dumps(out), flush=True)
    return 0


def _batched(args):
    """4096 CFGs: plain per-CFG two-pass form vs the batched form with exact
    two-pass sizing vs the batched form sized by the learned predictor."""
    import numpy as np
    import torch
    from paper_2210_16998_amd import cfggen, sizer, tpg

    cfgs = cfggen.c3_batch(4096)
    graphs = [tpg.load_cfg(c) for c in cfgs]
    model = sizer.DEFAULT_MODEL
    mlp = tpg.MLP.load(model) if os.path.exists(model) else None
    dev = tpg.TPG_OUT_DEVICE | tpg.TPG_NO_TIMING

    def timed(fn, reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - t) / reps, r

    def learned(ws):
        pred = mlp.forward(tpg.features(graphs))
        return tpg.batch_test_paths(graphs, ws=ws, flags=dev, predicted=pred)

    def twopass(ws):
        return tpg.batch_test_paths(graphs, ws=ws, flags=dev | tpg.TPG_FORCE_TWO_PASS)

    def onepass(ws):
        return tpg.batch_test_paths(graphs, ws=ws, flags=dev)

    res = {"workload": "4096 structured CFGs, vertices lognormal (median 40, clipped 10..300), "
                       "seeds 3000000+i"}
    ws = tpg.Workspace(0)
    twopass(ws)
    ms2, (r2, st2) = timed(lambda: twopass(ws), args.batch_reps)
    res["batched_two_pass_ms"] = ms2
    res["n_pp"] = int(st2["n_pp"])
    res["n_extensions"] = int(st2["n_extensions"])
    res["n_tp"] = int(st2["n_tp"])
    if mlp is not None:
        learned(ws)
        msl, (rl, stl) = timed(lambda: learned(ws), args.batch_reps)
        res["batched_learned_ms"] = msl
        res["prime_paths_per_s_learned"] = st2["n_pp"] / (msl * 1e-3)
        res["extensions_per_s_learned"] = st2["n_extensions"] / (msl * 1e-3)
        res["same_results_as_two_pass"] = bool(
            np.array_equal(rl.pp_first, r2.pp_first) and np.array_equal(rl.tp_first, r2.tp_first))
        res["gain_vs_batched_two_pass"] = ms2 / msl
        # cold start: fresh workspaces, predicted sizing vs growing by replay
        wc = tpg.Workspace(0)
        msc, (_, stc) = timed(lambda: learned(wc), 1)
        wc.close()
        wo = tpg.Workspace(0)
        mso, (_, sto) = timed(lambda: onepass(wo), 1)
        wo.close()
        res["cold_learned_ms"] = msc
        res["cold_learned_overflows"] = int(stc["n_overflows"])
        res["cold_unpredicted_ms"] = mso
        res["cold_unpredicted_overflows"] = int(sto["n_overflows"])
        res["over_allocation"] = stc["pred_nodes"] * 1.25 / max(1, stc["n_nodes"])
    ws1 = tpg.Workspace(0)
    t = time.perf_counter()
    n_plain = 0
    for g in graphs:
        _, tp, st = tpg.test_paths(g, ws=ws1, flags=dev | tpg.TPG_FORCE_TWO_PASS)
        n_plain += st["n_pp"]
    torch.cuda.synchronize()
    msp = 1000.0 * (time.perf_counter() - t)
    res["plain_per_cfg_two_pass_ms"] = msp
    assert n_plain == res["n_pp"]
    if "batched_learned_ms" in res:
        res["speedup_learned_vs_plain"] = msp / res["batched_learned_ms"]
    res["speedup_two_pass_batched_vs_plain"] = msp / ms2
    return res


if __name__ == "__main__":
    sys.exit(main())
