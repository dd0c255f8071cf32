"""Benchmark: exact prime paths + test paths of the 400-vertex stress CFG
(3 nested whiles, a 16-way switch, 60 if-else diamonds; 2.3e7 prime paths)
on one MI355X, with the ~200-vertex CFG, the 4096-CFG batch (plain, batched,
learned sizing) and the comparison variants as sub-objects.

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


def _copy_probe(mib: int) -> int:
    """One device-to-device copy of exactly `mib` MiB (torch's copy kernel),
    after three untimed ones: FETCH_SIZE / WRITE_SIZE read on it scale the
    counter readings of the path kernels."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(f"copied {mib} MiB in {ms:.3f} ms: {2 * mib / 1024 / (ms / 1e3):.0f} GiB/s "
          f"(read + write)", flush=True)
    return 0


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
    """Strongly connected components, prime-path types and the compositional
    method (Sec. 2, 2.1) on the benchmark CFG: the device SCC pass, the
    classification of its device-resident prime-path set (counts only), the
    component graph, the extraction, the internal prime paths of each
    component alone and the merge."""
    import torch
    from paper_2210_16998_amd import tpg
    g, rec = _workload()
    h = tpg.load_cfg(g)
    ws = tpg.Workspace(0)
    stream = torch.cuda.Stream()
    pp, _ = tpg.prime_paths(h, ws=ws, flags=tpg.TPG_OUT_DEVICE | tpg.TPG_NO_TIMING, stream=stream)
    out = {}
    f = tpg.TPG_OUT_DEVICE
    for name, fn in (("scc_ms", lambda: tpg.scc(h, ws=ws, stream=stream)),
                     ("types_ms", lambda: tpg.prime_path_types(h, pp, ws=ws, stream=stream,
                                                               want_types=False)),
                     ("ccfg_ms", lambda: tpg.ccfg(h, ws=ws, stream=stream)),
                     ("extraction_ms", lambda: tpg.scc_paths(h, ws=ws, flags=f, stream=stream)),
                     ("internal_ms", lambda: tpg.scc_internal_pps(h, ws=ws, flags=f,
                                                                  stream=stream)),
                     ("merge_ms", lambda: tpg.merged_pps(h, ws=ws, flags=f, stream=stream))):
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
        elif name == "types_ms":
            names = ["", "complete", "scc_internal", "scc_exit", "scc_entry", "other"]
            out["types"] = {names[t]: int(r[1][t]) for t in range(1, 6)}
        elif name == "ccfg_ms":
            out["n_ccfg_arcs"] = int(len(r[2]))
        elif name == "extraction_ms":
            out["extracted"] = {"entry_exit": len(r[0]), "exit": len(r[1]), "entry": len(r[2])}
        elif name == "internal_ms":
            out["n_internal"] = len(r)
        else:
            out["merged"] = {"complete": len(r[0]), "scc_exit": len(r[1]), "scc_entry": len(r[2])}
    ws.close()
    out["workload"] = (f"the benchmark CFG ({g.n} vertices, {out['n_components']} components): "
                       f"device SCC pass, the types of its {len(pp)} prime paths held on the "
                       f"device, the component graph, the extraction of Defs. 6-8, the internal "
                       f"prime paths of each component alone, and the merge of Sec. 2.1 (each call "
                       f"includes the graph upload and the SCC pass)")
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


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(g, threads: int, target_pp: int, seconds: float, chunk: int, seed: int):
    """The oracle over start-vertex chunks of `chunk` consecutive vertices, in
    a seeded random order, until `target_pp` prime paths are found (or
    `seconds` of prime-path work are spent); then its test-path stage
    (splice, sort, dedup) on the prime paths found.  Returns the timings and
    what was processed."""
    import numpy as np
    import oracle
    starts = np.random.default_rng(seed).permutation(np.arange(0, g.n, chunk))
    parts, done, t_pp = [], [], 0.0
    for s in starts:
        t = time.perf_counter()
        pl, _ = oracle.prime_paths_local(g, int(s), int(min(g.n, s + chunk)), nthreads=threads)
        t_pp += time.perf_counter() - t
        parts.append(pl)
        done.append(int(s))
        if sum(len(p) for p in parts) >= target_pp or t_pp >= seconds:
            break
    offs = [np.zeros(1, np.int64)]
    base = 0
    for pl in parts:
        offs.append(pl.offsets[1:] + base)
        base += int(pl.offsets[-1])
    pps = oracle.PathList(np.concatenate(offs), np.concatenate([pl.vertices for pl in parts]))
    t = time.perf_counter()
    tps, _ = oracle.test_paths(g, pps)
    t_tp = time.perf_counter() - t
    return {"n_pp": len(pps), "n_tp": len(tps), "pp_s": t_pp, "tp_s": t_tp,
            "starts": f"{len(done)} chunks of {chunk} start vertices (of {len(starts)}), "
                      f"seeded order"}


def _cpu_baseline(g, target_pp: int, seconds: float = 60.0):
    """The CPU oracle on a bounded sample of the same workload: DFS enumeration
    with the local prime test over start-vertex chunks taken in a seeded
    random order until about `target_pp` prime paths are found, then the
    test-path stage (splice, sort, dedup; one thread) on the prime paths
    found.  Run with the host threads a one-GPU job gets (at most 16) and
    with one thread."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(16, avail or 1))
    out = {"unit": "prime paths/s", "kind": "oracle", "cpu_model": _cpu_model(),
           "host_cpus_visible": avail}
    # both legs take the same start vertices (chunks of 16 in one seeded order)
    for name, th in (("all", threads), ("one_core", 1)):
        r = _oracle_sample(g, th, target_pp, seconds, 16, seed=17)
        rate = r["n_pp"] / (r["pp_s"] + r["tp_s"])
        rec = {"value": rate, "cores": th,
               "prime_paths_stage": {"seconds": r["pp_s"], "prime_paths_per_s": r["n_pp"] / r["pp_s"]},
               "test_paths_stage": {"seconds": r["tp_s"], "threads": 1,
                                    "prime_paths_per_s": r["n_pp"] / max(r["tp_s"], 1e-9)},
               "sample": f"{r['starts']}: {r['n_pp']} prime paths, {r['n_tp']} test paths; "
                         f"{r['pp_s'] + r['tp_s']:.1f} s"}
        if name == "all":
            out.update(rec)
        else:
            out["one_core"] = rec
    return out


def _whole_path(g, args, stream, copy_gbs: float, traffic_summary: str, pool_cap: int = 0):
    """Whole hot path (prime + test paths, device output) on graph g: a cold
    first call on a fresh workspace, `warmup` untimed steps, `steps` timed
    steps (level loop replayed from captured HIP graphs), then the same
    number of steps issued one launch at a time with a HIP event pair on the
    library's stream around every extension launch (the kernel's roofline)
    and per-phase events."""
    import torch
    from paper_2210_16998_amd import tpg
    h = tpg.load_cfg(g)
    ws = tpg.Workspace(0)
    flags = tpg.TPG_OUT_DEVICE

    def step(f=flags):
        return tpg.test_paths(h, ws=ws, flags=f, stream=stream, want_pp=True, pool_cap=pool_cap)

    torch.cuda.synchronize()
    t = time.perf_counter()
    step(flags | tpg.TPG_NO_TIMING)
    torch.cuda.synchronize()
    cold_ms = 1000.0 * (time.perf_counter() - t)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        step(flags | tpg.TPG_NO_TIMING)
        times.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    k_ms, k_launches, phases = 0.0, 0, []
    t2 = time.perf_counter()
    for _ in range(args.steps):
        _, _, st = step()
        k_ms += st["ms_extend_kernel"]
        k_launches += st["n_extend_launches"]
        phases.append(st)
    torch.cuda.synchronize()
    ms_timed = 1000.0 * (time.perf_counter() - t2) / args.steps
    n_pp, n_ext = st["n_pp"], st["n_extensions"]
    bpe = _bytes_per_extension(g.n)
    avg = k_ms / max(1, k_launches)
    per_launch = n_ext * bpe / max(1, st["n_extend_launches"])
    achieved = per_launch / (avg * 1e-3) / 1e9 if avg > 0 else 0.0

    # plain per-CFG two-pass form of the same graph, for context
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
    traffic = _measured_traffic(kname, traffic_summary)
    dev_bytes = st["device_bytes"]
    ws.close()
    measured = traffic / (avg * 1e-3) / 1e9 if traffic and avg > 0 else None
    return {
        "ms_per_step": ms, "n_pp": n_pp, "n_extensions": n_ext, "n_tp": st["n_tp"],
        "n_tp_spliced": st["n_tp_spliced"], "levels": st["n_levels"],
        "prime_paths_per_s": n_pp / (ms * 1e-3), "extensions_per_s": n_ext / (ms * 1e-3),
        "test_paths_per_s": st["n_tp"] / (ms * 1e-3),
        "step_ms": {"median": 1000.0 * statistics.median(times),
                    "mean": 1000.0 * statistics.fmean(times),
                    "kernel_timed_pass_mean": ms_timed, "cold_first_call": cold_ms},
        "phase_ms_median": {"extend": med("ms_extend"), "rank_materialize": med("ms_rank"),
                            "test_paths": med("ms_tp"), "total_device": med("ms_total"),
                            "extend_kernel": med("ms_extend_kernel")},
        "plain_two_pass_ms_per_step": ms_plain,
        "device_bytes": dev_bytes,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "measured_GBps": measured,
                     "measured_frac": measured / HBM_PEAK_GBS if measured else None,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "algorithmic_bytes_per_launch": per_launch, "bytes_per_extension": bpe,
                     "launches_per_step": st["n_extend_launches"], "avg_launch_ms": avg},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-pp", type=int, default=600_000,
                    help="prime paths in each bounded oracle sample")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-cfg209", action="store_true")
    ap.add_argument("--no-paper-form", action="store_true")
    ap.add_argument("--no-covering", action="store_true")
    ap.add_argument("--no-components", action="store_true")
    ap.add_argument("--no-prior-schedule", action="store_true")
    ap.add_argument("--only", choices=["batched", "batched_learned", "paper_form", "covering",
                                       "components", "prior_schedule"],
                    help="run one section alone and print its JSON (for profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (the reference "
                         "traffic that scales HBM counter readings) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        return _copy_probe(args.copy_probe)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path is "
              f"single-GPU", file=sys.stderr)
        return 2

    import torch
    from paper_2210_16998_amd import cfggen

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.only:
        fn = {"batched": _batched, "batched_learned": _batched_learned_only,
              "paper_form": _paper_form, "covering": _covering,
              "components": _components, "prior_schedule": _prior_schedule}[args.only]
        print(json.dumps({args.only: fn(args)}), flush=True)
        return 0
    stream = torch.cuda.Stream()
    copy_gbs = _copy_peak(stream)
    g = cfggen.c5_cfg()
    cap = 64 << 30  # the stress workload's pool cap (64 GiB of HBM)
    r = _whole_path(g, args, stream, copy_gbs, "k_extend_stress400_hbm_traffic.md", pool_cap=cap)
    out = {
        "metric": METRIC,
        "value": r["prime_paths_per_s"],
        "unit": "prime paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"stress CFG, {g.n} vertices, {g.n_edges} arcs, cyclomatic "
                               f"{g.cyclomatic} (3 nested whiles, 16-way switch, 60 if-else "
                               f"diamonds); whole path: prime + test paths",
                   "n_pp": r["n_pp"], "n_extensions": r["n_extensions"], "n_tp": r["n_tp"],
                   "levels": r["levels"], "pool_cap_bytes": cap},
    }
    out["roofline"] = r.pop("roofline")
    for k in ("extensions_per_s", "test_paths_per_s", "n_tp_spliced", "step_ms",
              "phase_ms_median", "plain_two_pass_ms_per_step", "device_bytes"):
        out[k] = r[k]
    if not args.no_cfg209:
        g2, rec = _workload()
        r2 = _whole_path(g2, args, stream, copy_gbs, "k_extend_cfg209_hbm_traffic.md")
        r2["workload"] = (f"single structured CFG, {g2.n} vertices, {g2.n_edges} arcs, "
                          f"cyclomatic {g2.cyclomatic}, seed {rec['seed']} (prime + test paths)")
        out["cfg209"] = r2
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
        out["cpu_baseline"] = _cpu_baseline(g, args.cpu_pp)
        if "cfg209" in out:
            out["cfg209"]["cpu_baseline"] = _cpu_baseline(_workload()[0], args.cpu_pp // 2)
    print(json.dumps(out), flush=True)
    return 0


def _batched_learned_only(args):
    """The batched call sized by the learned predictor alone, warm (two
    untimed calls, then batch_reps timed ones), planned on the host each
    time and then replayed as one graph: what a kernel profile of that form
    is taken on."""
    import torch
    from paper_2210_16998_amd import cfggen, sizer, tpg, tuning
    graphs = [tpg.load_cfg(c) for c in cfggen.c3_batch(4096)]
    mlp = tpg.MLP.load(sizer.DEFAULT_MODEL)
    ws = tpg.Workspace(0)
    if tuning.load(ws) is None:
        tpg.autotune(graphs, ws)
    dev = tpg.TPG_OUT_DEVICE | tpg.TPG_NO_TIMING
    out = {}
    # every call planned on the host, then the same call replayed as one graph
    for name, flags in (("batched_learned_ms", dev | tpg.TPG_NO_CALL_GRAPH),
                        ("batched_learned_replayed_ms", dev)):
        def call():
            return tpg.batch_test_paths(graphs, ws=ws, flags=flags,
                                        predicted=mlp.forward(tpg.features(graphs)))
        call()
        call()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.batch_reps):
            _, st = call()
        torch.cuda.synchronize()
        out[name] = 1000.0 * (time.perf_counter() - t) / args.batch_reps
        out[name.replace("_ms", "_call_graph")] = int(st["call_graph"])
    out.update({"n_pp": int(st["n_pp"]), "n_unions": int(st["n_unions"]),
                "n_overflows": int(st["n_overflows"])})
    return out


def _batched(args):
    """4096 CFGs: plain per-CFG two-pass form vs the batched form with exact
    two-pass sizing vs the batched form sized by the learned predictor."""
    import numpy as np
    import torch
    from paper_2210_16998_amd import cfggen, sizer, tpg, tuning

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

    # ordinary calls (launches planned on the host every time); the *_replayed
    # figures repeat the same call, which then runs as one captured graph
    plan = tpg.TPG_NO_CALL_GRAPH

    def learned(ws, extra=plan):
        pred = mlp.forward(tpg.features(graphs))
        return tpg.batch_test_paths(graphs, ws=ws, flags=dev | extra, predicted=pred)

    def twopass(ws):
        return tpg.batch_test_paths(graphs, ws=ws, flags=dev | tpg.TPG_FORCE_TWO_PASS)

    def onepass(ws, extra=plan):
        return tpg.batch_test_paths(graphs, ws=ws, flags=dev | extra)

    def snapshot(r):
        """Copies of a device result's arrays (the next call on the same
        workspace overwrites them)."""
        po, pv = r.pp.torch_views()
        to, tv = r.tp.torch_views()
        return [x.clone() for x in (po, pv, to, tv)] + [r.pp_first.copy(), r.tp_first.copy()]

    def same(a, b):
        return all((torch.equal(x, y) if torch.is_tensor(x) else np.array_equal(x, y))
                   for x, y in zip(a, b))

    res = {"workload": "4096 structured CFGs, vertices lognormal (median 40, clipped 10..300), "
                       "seeds 3000000+i"}
    ws = tpg.Workspace(0)
    # launch shapes of the extension kernel per visited-set width: the cached
    # autotuner result for this GPU, else tuned now on this batch
    shape = tuning.load(ws)
    if shape is None:
        t = time.perf_counter()
        shape = tpg.autotune(graphs, ws)
        res["tuning"] = {"source": "autotuned on this batch",
                         "seconds": time.perf_counter() - t, **shape}
    else:
        res["tuning"] = {"source": "cache " + os.path.relpath(tuning.DEFAULT_CACHE, ROOT), **shape}
    shape = tpg.get_tuning(ws)

    def fresh():
        w = tpg.Workspace(0)
        tpg.set_tuning(w, shape)
        return w

    twopass(ws)
    ms2, (r2, st2) = timed(lambda: twopass(ws), args.batch_reps)
    ref = snapshot(r2)
    res["batched_two_pass_ms"] = ms2
    res["n_pp"] = int(st2["n_pp"])
    res["n_extensions"] = int(st2["n_extensions"])
    res["n_tp"] = int(st2["n_tp"])
    onepass(ws)
    ms1, (r1, _) = timed(lambda: onepass(ws), args.batch_reps)
    res["batched_one_pass_unpredicted_ms"] = ms1
    res["one_pass_same_paths_as_two_pass"] = same(snapshot(r1), ref)
    onepass(ws, 0)
    onepass(ws, 0)
    ms1r, (r1r, st1r) = timed(lambda: onepass(ws, 0), args.batch_reps)
    res["batched_one_pass_replayed_ms"] = ms1r
    res["one_pass_replayed_call_graph"] = int(st1r["call_graph"])
    res["one_pass_replayed_same_paths_as_two_pass"] = same(snapshot(r1r), ref)
    if mlp is not None:
        learned(ws)
        msl, (rl, stl) = timed(lambda: learned(ws), args.batch_reps)
        res["batched_learned_ms"] = msl
        res["prime_paths_per_s_learned"] = st2["n_pp"] / (msl * 1e-3)
        res["extensions_per_s_learned"] = st2["n_extensions"] / (msl * 1e-3)
        # every offset and vertex of both path sets, not only the counts
        res["same_paths_as_two_pass"] = same(snapshot(rl), ref)
        res["gain_vs_batched_two_pass"] = ms2 / msl
        res["gain_vs_batched_one_pass_unpredicted"] = ms1 / msl
        learned(ws, 0)
        learned(ws, 0)
        mslr, (rlr, stlr) = timed(lambda: learned(ws, 0), args.batch_reps)
        res["batched_learned_replayed_ms"] = mslr
        res["learned_replayed_call_graph"] = int(stlr["call_graph"])
        res["learned_replayed_same_paths_as_two_pass"] = same(snapshot(rlr), ref)
        # cold start: fresh workspaces, predicted sizing vs growing by replay
        wc = fresh()
        msc, (_, stc) = timed(lambda: learned(wc), 1)
        wc.close()
        wo = fresh()
        mso, (_, sto) = timed(lambda: onepass(wo), 1)
        wo.close()
        res["cold_learned_ms"] = msc
        res["cold_learned_overflows"] = int(stc["n_overflows"])
        res["cold_unpredicted_ms"] = mso
        res["cold_unpredicted_overflows"] = int(sto["n_overflows"])
        res["cold_gain"] = mso / msc
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
