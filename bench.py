#!/usr/bin/env python3
"""Top-k closeness benchmark on one MI355X.

Default workload: the learned-ordering configuration at scale, the
collaboration projection of 2,000,000 actors onto 500,000 groups (Zipf(2.1)
group sizes capped at 200, seed 4; 40M arcs), k = 10.  One step = the top-k
query (every k the workload is queried with) on a graph already resident in
HBM.  `value` is the batched mode with the learned source order (the order
perceptron's k best-scored sources, then the grouped degree order), in the
batch width and deferral the workload is tuned for.

Throughput is GTEPS: visited arcs divided by the wall time of the step.  Where
the oracle's sequential run in decreasing-degree order is stored with the
expected results (BA, R-MAT, RGG 2^18), its m_vis is the fixed work numerator
of every variant; on the 2M-actor graph, where that run takes days, the
numerator is the GPU's own count of the arcs each source's search scans
(``work_kind`` in the line says which).

The JSON line also carries: the same batched mode with the grouped degree
order (the method without the learned part), the plain comparator (one batch
of 64 sources per host-loop iteration, degree order; on BA n = 1M when the
workload is too large for it, next to batched+learned on that graph), the
roofline of the persistent level kernel (algorithmic bytes over its HIP-event
time, and the measured HBM traffic from the committed counter profile), the
CPU oracle timed on the host cores on a bounded sample, and the parity of the
timed configuration against the oracle's stored answers.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "top-k closeness wall time & GTEPS on 1 MI355X; batched+learned vs plain"
HBM_PEAK_GBS = 8000.0
# batched-mode width and deferral budget per workload, from measured sweeps
# (same answers for every setting): hub-dominated BA favours 64-source batches
# with deep sources deferred; R-MAT and the clique-rich collaboration graph
# favour 256-source batches, the latter with no deferral (7.3 s vs 11.9 s)
WORKLOAD_KNOBS = {"ba1m": (64, 0), "ba2k": (64, 0), "rmat21": (256, 0), "collab": (256, -1), "rgg": (256, 0),
                  "rgg18": (256, 0), "collab500k": (256, -1), "rgg20": (256, 0)}
# geometric graphs have no hubs: batches of nearby sources share their levels
WORKLOAD_ORDER = {"rgg": "locality", "rgg18": "locality", "rgg20": "locality"}
# where the full-size graph has no stored oracle answer, the same family at
# the largest size the oracle finishes checks the timed configuration
PARITY_PROXY = {"collab": "collab500k", "rgg": "rgg20"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(arcs: int, entries: int, discovered: int, W: int, trial: bool = True) -> int:
    """Minimal HBM bytes of the level work of the persistent kernel:
    per scanned arc: col[e] (4 B) + seen[w] gather (W/8 B), plus deg[col[e]]
    (4 B) in the W = 64 kernel, whose over-counted bound test (trial) sums the
    degree of every arc's target;
    per expanded frontier entry: list entry (4 B) + row_ptr pair (8 B) + cur[u] (W/8 B);
    per discovered entry of an exactly counted level: list entry (4 B) + deg (4 B)
    + nxt read+reset (2 W/8 B) + seen read+write (2 W/8 B) + cur write (W/8 B)."""
    wb = W // 8
    return arcs * ((8 if trial else 4) + wb) + entries * (12 + wb) + discovered * (8 + 5 * wb)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when there is none or the kernel
    source has changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_{workload}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    info = json.loads(m.group(1))
    if device_source_hash() != info.get("device_source_sha256_16"):
        return None
    return info.get("traffic_bytes_per_launch")


def device_source_hash() -> str:
    """SHA-256 (16 hex digits) of the device part of csrc/topk.hip: all of the
    file above its host-side marker, where every kernel and device function
    of the level step lives.  Host-side edits below the marker leave it
    unchanged; any kernel edit changes it."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1507_01490_amd", "csrc", "topk.hip")).read()
    mark = "// --------------------------------------------------------- host side"
    if src.count(mark) != 1:
        return ""
    return hashlib.sha256(src.split(mark)[0].encode()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="collab",
                    help="collab (default: 2M actors), ba1m, ba2k, rmat21, rgg, rgg18, rgg20, collab500k, serve512, "
                         "scaling or snapshots")
    ap.add_argument("--mode", default="batched", choices=["batched", "plain"])
    ap.add_argument("--width", type=int, default=0, help="sources per batch (0: the workload's default)")
    ap.add_argument("--defer-arcs", type=int, default=None,
                    help="batched mode: deferral budget in arcs (-1 never; default: the workload's)")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--order", default="auto",
                    choices=["auto", "degree", "grouped", "locality", "learned", "learned_grouped", "learned_locality"],
                    help="source order of the timed mode (auto: the learned order, i.e. the perceptron's k best-scored "
                         "sources, then the grouped degree order, or the locality order on geometric graphs)")
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="timed steps of the plain comparator (0 = skip; default 1; on workloads too large for it "
                         "(collab, rgg) it runs on BA n = 1M instead, next to batched+learned there)")
    ap.add_argument("--grouped-steps", type=int, default=2,
                    help="timed steps of the batched mode without the learned order (grouped degree order, or "
                         "locality on geometric graphs; 0 = skip)")
    ap.add_argument("--queue", type=int, default=0, choices=[0, 1],
                    help="serve512: continuous batching through the device queue of one running kernel")
    ap.add_argument("--mix-count", type=int, default=512, help="serve512: graphs in the mix")
    ap.add_argument("--mix-max-n", type=float, default=2e5, help="serve512: largest graph size of the mix")
    ap.add_argument("--request-timeout", type=int, default=120, help="serve512: seconds before a request is an error")
    ap.add_argument("--footnote", type=int, default=0, choices=[0, 1],
                    help="undirected footnote bound of Section 2.3 in the timed mode (same answer)")
    ap.add_argument("--tune", type=int, default=0, choices=[0, 1],
                    help="pick the batched-mode knobs per k with the autotuner (bc_autotune) before the timed "
                         "region (tuning time reported, not timed)")
    ap.add_argument("--trial", type=int, default=1, choices=[0, 1],
                    help="over-counted bound test before exact level counts in the persistent kernel (same answer)")
    ap.add_argument("--big-scc", type=int, default=1, choices=[0, 1],
                    help="directed workloads: largest-SCC refinement of the reach bounds (Section 2.4; same "
                         "answer); ignored on undirected graphs")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--sample-check", type=int, default=16,
                    help="full-size graphs without a stored answer: seeded nodes checked to rank below the k-th")
    ap.add_argument("--lanes", type=int, default=None,
                    help="serve512: lanes (default 4; 1 with --queue 1, where the lanes only prepare requests and "
                         "one preparing thread measured fastest: 48 requests in 0.44 s, against 5.9 s with 3)")
    ap.add_argument("--serve-slots", type=int, default=64, help="serve512: workgroups per persistent kernel")
    ap.add_argument("--budget-mb", type=int, default=2048, help="serve512: device memory budget")
    ap.add_argument("--load", type=float, default=0.8, help="serve512: Poisson rate as a fraction of capacity")
    ap.add_argument("--family-knobs", type=int, default=1, choices=[0, 1],
                    help="serve512: per-family request options (grids: W=256, locality order, no deferral)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale reference for HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "launches": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "sharding sources over several GPUs is designed but not implemented, so no multi-GPU figure exists.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1507_01490_amd as bc
    from paper_1507_01490_amd import workloads

    if args.workload == "serve512":
        serve_bench(args, bc, workloads)
        return
    if args.workload == "scaling":
        scaling_bench(args, bc)
        return
    if args.workload == "snapshots":
        snapshot_bench(args, bc)
        return

    wdef, ddef = WORKLOAD_KNOBS.get(args.workload, (64, 0))
    if args.width == 0:
        args.width = wdef
    if args.defer_arcs is None:
        args.defer_arcs = ddef
    base_order = WORKLOAD_ORDER.get(args.workload, "grouped")  # the method's own order for this family
    if args.order == "auto":
        args.order = "learned_locality" if base_order == "locality" else "learned_grouped"
    too_big_for_plain = args.workload in ("collab", "rgg", "rgg18", "rgg20", "collab500k")
    if args.plain_steps is None:
        args.plain_steps = 1
    t0 = time.time()
    g = workloads.build(args.workload)
    log(f"[bench] built {args.workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    gold = load_gold(args.workload, g)
    ks = list(workloads.KS[args.workload])

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    G = bc.Graph(rp, col, directed=g.directed, stream=stream, big_scc=bool(args.big_scc))
    del rp, col
    log(f"[bench] graph resident on GPU, pre-processing {G.preprocess_ms:.1f} ms")

    tuned, tune_s = {}, 0.0
    if args.tune and args.mode == "batched":
        tt = time.perf_counter()
        for k in ks:
            tuned[k], rep = G.autotune(k, repeats=1, width=args.width, defer_arcs=args.defer_arcs)
            log(f"[bench] autotune k={k}: {tuned[k]} ({rep})")
        tune_s = time.perf_counter() - tt

    def knobs(order):
        return dict(mode=args.mode, width=args.width, slots=args.slots, order=order, footnote=bool(args.footnote),
                    trial=bool(args.trial), defer_arcs=args.defer_arcs)

    def step(mode, order=args.order, footnote=bool(args.footnote)):
        if mode == "batched" and tuned:
            return [G.topk(k, footnote=footnote, trial=bool(args.trial), **tuned[k]) for k in ks]
        if mode == "plain":  # the comparator: one 64-source batch per host-loop iteration
            return [G.topk(k, mode="plain", width=64, order=order, footnote=footnote) for k in ks]
        return [G.topk(k, **knobs(order)) for k in ks]

    for i in range(args.warmup):
        step(args.mode)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    def width_of(k):
        return tuned[k]["width"] if tuned else args.width

    agg = dict(persistent_ms=0.0, seed_ms=0.0, defer_ms=0.0, n_deferred=0, arcs=0, entries=0, disc=0, m_vis=0,
               alg_bytes=0,
               node_arcs=0, levels=0, lds_levels=0, record_levels=0, spills=0, record_ms=0.0, record_arcs=0,
               phase_ms=[0.0] * 5)
    parity = True if gold is not None else None  # None: no stored oracle answer for this graph
    t_start = time.perf_counter()
    for i in range(args.steps):
        out = step(args.mode)
        for k, r in zip(ks, out):
            s = r.stats
            agg["alg_bytes"] += algorithmic_bytes(s["persistent_arcs"], s["persistent_entries"],
                                                  s["persistent_discovered"], width_of(k),
                                                  trial=width_of(k) == 64 and bool(args.trial))
            agg["persistent_ms"] += s["persistent_ms"]
            agg["seed_ms"] += s["seed_ms"]
            agg["defer_ms"] += s["defer_ms"]
            agg["n_deferred"] += s["n_deferred"]
            agg["arcs"] += s["persistent_arcs"]
            agg["entries"] += s["persistent_entries"]
            agg["disc"] += s["persistent_discovered"]
            agg["m_vis"] += s["m_vis"]
            agg["node_arcs"] += s["node_arcs"]
            agg["levels"] += s["levels"]
            for key in ("lds_levels", "record_levels", "spills", "record_ms", "record_arcs"):
                agg[key] += s[key]
            agg["phase_ms"] = [a + b for a, b in zip(agg["phase_ms"], s["phase_ms"])]
        c = check(gold, ks, out)
        if parity is not None:
            parity = parity and bool(c)
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    log(f"[bench] {args.mode} ({args.order}): {ms_per_step:.2f} ms/step, parity={parity}")

    if gold is not None and all("m_vis_seq" in gold["results"][str(k)] for k in ks):
        work = sum(gold["results"][str(k)]["m_vis_seq"] for k in ks)
        work_kind = "oracle m_vis, sequential run in decreasing-degree order (stored with the expected results)"
    else:
        work = agg["m_vis"] // args.steps
        work_kind = "GPU-counted m_vis of the timed run (arcs each source's search scans, summed over sources)"
    gteps = work / (ms_per_step / 1e3) / 1e9

    # the same batched mode without the learned order
    grouped = None
    if args.grouped_steps > 0 and args.mode == "batched" and not tuned and args.order != base_order:
        step("batched", base_order)
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for _ in range(args.grouped_steps):
            gout = step("batched", base_order)
        torch.cuda.synchronize()
        gms = (time.perf_counter() - tg0) * 1e3 / args.grouped_steps
        grouped = dict(ms_per_step=round(gms, 3), value=round(work / (gms / 1e3) / 1e9, 4), unit="GTEPS",
                       order=base_order, parity=check(gold, ks, gout),
                       m_vis_gpu=sum(r.stats["m_vis"] for r in gout),
                       learned_speedup=round(gms / ms_per_step, 4))
        log(f"[bench] batched ({base_order}): {gms:.1f} ms/step")

    # the timed configuration on the oracle-sized member of the same family
    parity_proxy = None
    proxy = PARITY_PROXY.get(args.workload)
    if proxy is not None and args.mode == "batched" and not tuned:
        pg = workloads.build(proxy)
        pgold = load_gold(proxy, pg)
        if pgold is not None:
            with bc.Graph(pg.row_ptr, pg.col, directed=pg.directed) as PG:
                pks = list(workloads.KS[proxy])
                pout = [PG.topk(k, **knobs(args.order)) for k in pks]
                parity_proxy = dict(workload=workloads.DESCRIPTION[proxy], parity=check(pgold, pks, pout),
                                    order=args.order, width=args.width, defer_arcs=args.defer_arcs)
            log(f"[bench] parity on {proxy}: {parity_proxy['parity']}")
        del pg

    # full size, no stored answer: each returned node's exact reach and
    # farness by one oracle BFS, and a seeded sample that must rank below
    sampled = None
    if gold is None and args.sample_check > 0 and args.workload in ("collab", "rgg"):
        sampled = sampled_check(g, out[0], args.sample_check)
        log(f"[bench] sampled full-size check: {sampled}")

    plain = None
    if args.plain_steps > 0 and args.mode != "plain":
        if not too_big_for_plain:
            step("plain", "degree", False)  # plain-mode workspace already sized; one untimed pass
            torch.cuda.synchronize()
            tp0 = time.perf_counter()
            for _ in range(args.plain_steps):
                pout = step("plain", "degree", False)
            torch.cuda.synchronize()
            pms = (time.perf_counter() - tp0) * 1e3 / args.plain_steps
            plain = dict(ms_per_step=round(pms, 3), value=round(work / (pms / 1e3) / 1e9, 4), unit="GTEPS",
                         parity=check(gold, ks, pout), speedup_of_value=round(pms / ms_per_step, 2),
                         config="one batch of 64 sources per host-loop iteration, degree order")
            log(f"[bench] plain: {pms:.1f} ms/step, batched speed-up {pms / ms_per_step:.2f}x")
        else:
            plain = plain_on_ba1m(args, bc, workloads, torch)

    roofline = None
    widths = sorted({width_of(k) for k in ks})
    kernel = "k_batched_lds<1>" if widths == [64] else (f"k_batched<{widths[0] // 64}>" if len(widths) == 1 else
                                                        "k_batched_lds<1>/k_batched<WW>")
    if args.mode == "batched" and agg["persistent_ms"] > 0:
        nlaunch = args.steps * len(ks)
        bytes_per_launch = agg["alg_bytes"] / nlaunch
        avg_ms = agg["persistent_ms"] / nlaunch
        achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=measured_traffic(kernel, args.workload),
                        kernel=kernel, avg_launch_ms=round(avg_ms, 4),
                        bytes_per_launch=int(bytes_per_launch),
                        arcs_per_launch=int(agg["arcs"] / nlaunch))

    cpu = None
    if not args.skip_cpu:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        sample = workloads.cpu_sample(args.workload)
        if sample is not None or gold is not None:
            tc0 = time.perf_counter()
            if sample is None:
                for k in ks:
                    oracle.topk(g, k, nthreads=threads)
                cwork, what = work, f"the full step (k={','.join(map(str, ks))}) on the same graph"
            else:
                sg, what = sample
                cwork = sum(oracle.topk(sg, k, nthreads=threads)["stats"]["m_vis"] for k in ks)
                what = f"k={','.join(map(str, ks))} on {what}; m_vis {cwork}"
            tc = time.perf_counter() - tc0
            cpu = dict(value=round(cwork / tc / 1e9, 4), unit="GTEPS", cores=threads, kind="oracle",
                       sample=f"{what}, {threads} threads, {tc:.1f} s")
            log(f"[bench] cpu oracle: {tc:.1f}s with {threads} threads")

    line = dict(metric=METRIC, value=round(gteps, 4), unit="GTEPS", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(ms_per_step, 3), higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="int64", data="synthetic",
                config=dict(workload=workloads.DESCRIPTION[args.workload], k=ks, mode=args.mode,
                            width=args.width, defer_arcs=args.defer_arcs, order=args.order,
                            footnote=bool(args.footnote),
                            trial=bool(args.trial),
                            tuned={str(k): v for k, v in tuned.items()} if tuned else None,
                            tune_s=round(tune_s, 2) if tuned else None,
                            big_scc=bool(args.big_scc), parity_vs_oracle=parity if gold is not None else
                            (parity_proxy["parity"] if parity_proxy else None),
                            work_m_vis=int(work), work_kind=work_kind),
                parity_detail=dict(stored_answer_full_size=parity, same_config_oracle_sized_graph=parity_proxy,
                                   sampled_full_size=sampled),
                breakdown_ms_per_step=dict(seed=round(agg["seed_ms"] / args.steps, 3),
                                           persistent=round(agg["persistent_ms"] / args.steps, 3),
                                           deferred=round(agg["defer_ms"] / args.steps, 3),
                                           n_deferred=agg["n_deferred"] // args.steps,
                                           node_arcs=agg["node_arcs"] // args.steps,
                                           m_vis_gpu=agg["m_vis"] // args.steps),
                persistent_detail=dict(
                    lds_levels=agg["lds_levels"] // args.steps, record_levels=agg["record_levels"] // args.steps,
                    spills=agg["spills"] // args.steps, record_arcs=agg["record_arcs"] // args.steps,
                    workgroup_ms_record=round(agg["record_ms"] / args.steps, 1),
                    workgroup_ms_phases=dict(zip(("setup", "count", "cut", "build", "reset"),
                                                 [round(x / args.steps, 1) for x in agg["phase_ms"]]))),
                roofline=roofline, cpu_baseline=cpu, batched_without_learned=grouped, plain=plain)
    print(json.dumps(line), flush=True)
    G.close()


def load_gold(name, g):
    """The oracle's stored answer for workload `name` if it is on this very
    graph (same SHA-256 of the CSR), else None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        gold = json.load(f)
    if gold["sha256"] != g.sha256():
        log(f"[bench] WARNING: generated {name} differs from the stored one; parity not checked")
        return None
    return gold


def check(gold, ks, results):
    """Results equal the stored oracle answer element by element (None: no answer)."""
    if gold is None:
        return None
    ok = True
    for k, res in zip(ks, results):
        ref = gold["results"][str(k)]
        ok = ok and res.ids.tolist() == ref["ids"] and [int(x) for x in res.farness] == ref["farness"] \
            and [int(x) for x in res.reach] == ref["reach"]
    return ok


def sampled_check(g, res, count):
    """Exact (r, f) of every returned node by one oracle BFS each, the keys in
    decreasing order, and `count` seeded non-isolated nodes outside the
    result, each of which must rank below the returned k-th node."""
    import numpy as np

    import oracle

    def exact(v):
        d = oracle.bfs(g, int(v)).astype(np.int64)
        reached = d >= 0
        return int(reached.sum()), int(d[reached].sum())

    t0 = time.perf_counter()
    ok = all(exact(v) == (int(r), int(f)) for v, f, r in zip(res.ids, res.farness, res.reach))
    keys = [oracle.closeness_key(r, f) for r, f in zip(res.reach, res.farness)]
    for i in range(len(keys) - 1):
        ok = ok and (keys[i] > keys[i + 1] or (keys[i] == keys[i + 1] and res.ids[i] < res.ids[i + 1]))
    kth_key, kth_id = keys[-1], int(res.ids[-1])
    rng = np.random.default_rng(12)
    cand = np.flatnonzero(np.diff(g.row_ptr) > 0)
    top = set(res.ids.tolist())
    sample = [int(v) for v in rng.choice(cand, 2 * count, replace=False) if int(v) not in top][:count]
    for v in sample:
        r, f = exact(v)
        kv = oracle.closeness_key(r, f)
        ok = ok and (kv < kth_key or (kv == kth_key and v > kth_id))
    return dict(ok=bool(ok), returned_checked=len(res.ids), sampled_below_kth=len(sample),
                seconds=round(time.perf_counter() - t0, 1))


def plain_on_ba1m(args, bc, workloads, torch):
    """The plain comparator where the workload is too large for it: BA n = 1M,
    k = 1, 10, 100, plain (one 64-source batch per host-loop iteration, degree
    order) next to batched+learned on the same graph, both checked against
    the stored oracle answer."""
    g = workloads.build("ba1m")
    gold = load_gold("ba1m", g)
    ks = list(workloads.KS["ba1m"])
    w, d = WORKLOAD_KNOBS["ba1m"]
    with bc.Graph(g.row_ptr, g.col) as G:
        def run(**kw):
            return [G.topk(k, **kw) for k in ks]
        lk = dict(mode="batched", width=w, defer_arcs=d, order="learned_grouped")
        run(**lk)
        run(mode="plain", width=64, order="degree")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lout = run(**lk)
        t1 = time.perf_counter()
        pout = run(mode="plain", width=64, order="degree")
        t2 = time.perf_counter()
    lms, pms = (t1 - t0) * 1e3, (t2 - t1) * 1e3
    work = sum(gold["results"][str(k)]["m_vis_seq"] for k in ks) if gold else None
    out = dict(workload=workloads.DESCRIPTION["ba1m"], k=ks, plain_ms_per_step=round(pms, 3),
               batched_learned_ms_per_step=round(lms, 3), speedup=round(pms / lms, 2),
               plain_parity=check(gold, ks, pout), batched_learned_parity=check(gold, ks, lout),
               config="plain: one batch of 64 sources per host-loop iteration, degree order; batched+learned: "
                      "W = 64, persistent kernel, learned head + grouped tail")
    if work:
        out.update(plain_gteps=round(work / (pms / 1e3) / 1e9, 4), batched_learned_gteps=round(work / (lms / 1e3) / 1e9, 4))
    log(f"[bench] plain on ba1m: {pms:.1f} ms/step vs batched+learned {lms:.1f} ms/step")
    return out


def scaling_bench(args, bc):
    """The paper's machine-independent measures on seeded synthetic families of
    growing size (Section 4): the performance ratio m_vis / (m n) of the
    sequential-equivalent visited arcs the GPU counts, its inverse against n
    (which the paper finds close to linear on its growing actor graph, i.e.
    a running time close to O(m)), and the positive race: how much m_vis
    grows when the k-th record is shared by many concurrent searches (the
    batched mode, up to ~16k sources in flight) instead of one batch of 64 at
    a time (the plain mode), both in decreasing-degree order.  The GPU's m_vis
    counter itself is pinned to the oracle's by a test (no cut: k = n)."""
    import numpy as np
    import torch
    from paper_1507_01490_amd import synth
    torch.cuda.set_device(0)
    families = {
        "ba": lambda n, s: synth.barabasi_albert(n, 5, s),
        "er": lambda n, s: synth.erdos_renyi(n, 8.0, s),
        "collab": lambda n, s: synth.collaboration(4 * n, n, 2.1, 200, s),
    }
    sizes = {"ba": [1 << e for e in range(12, 21, 2)], "er": [1 << e for e in range(12, 21, 2)],
             "collab": [1 << e for e in range(12, 17, 2)]}
    rows = []
    for fam, make in families.items():
        for n in sizes[fam]:
            g = make(n, 7)
            with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
                for k in (1, 10):
                    # the race compares the two modes in one order (the paper's
                    # degree order), so that it measures only how stale the
                    # k-th record is when many searches share it
                    rb = G.topk(k, mode="batched", order="degree")
                    rg = G.topk(k, mode="batched")
                    rp = G.topk(k, mode="plain", order="degree") if n <= (1 << 16) else None
                    mn = float(G.m) * float(G.n)
                    row = dict(family=fam, n=G.n, m=G.m, k=k, ratio_batched=rb.stats["m_vis"] / mn,
                               ratio_batched_grouped=rg.stats["m_vis"] / mn,
                               ms_batched=round(rb.stats["query_ms"], 2), ms_batched_grouped=round(rg.stats["query_ms"], 2))
                    assert rg.ids.tolist() == rb.ids.tolist()
                    if rp is not None:
                        row["ratio_plain"] = rp.stats["m_vis"] / mn
                        row["race"] = rb.stats["m_vis"] / max(rp.stats["m_vis"], 1) - 1.0
                        assert rp.ids.tolist() == rb.ids.tolist()
                    rows.append(row)
                    log(f"[scaling] {fam} n={G.n} k={k} ratio={row['ratio_batched']:.3e} "
                        f"race={row.get('race', float('nan')):.3f} {row['ms_batched']} ms")
    fits = {}
    for fam in families:
        for k in (1, 10):
            pts = [(r["n"], 1.0 / r["ratio_batched"]) for r in rows if r["family"] == fam and r["k"] == k]
            x = np.array([p[0] for p in pts], float)
            y = np.array([p[1] for p in pts], float)
            c = np.polyfit(x, y, 1)
            r2 = 1.0 - ((y - np.polyval(c, x)) ** 2).sum() / max(((y - y.mean()) ** 2).sum(), 1e-300)
            fits[f"{fam}_k{k}"] = dict(slope=c[0], intercept=c[1], r2=round(float(r2), 4))
    print(json.dumps(dict(metric="performance ratio m_vis/(m n) and positive race on 1 MI355X", rows=rows,
                          inverse_ratio_linear_fit=fits, data="synthetic",
                          config=dict(workload="BA m=5 and ER avg deg 8 at n = 2^12 .. 2^20; collaboration with n "
                                               "groups of Zipf(2.1) sizes over 4n actors, n = 2^12 .. 2^16; seed 7; "
                                               "plain-mode comparison up to 2^16", k=[1, 10]))), flush=True)


def snapshot_bench(args, bc):
    """A growing collaboration graph (the shape of the paper's actor-graph
    case study on synthetic data): 16 snapshots, k = 10 on each.  Cold: the
    grouped degree order.  Warm: the previous snapshot's top-k first
    (opts.first), then the same order.  Both must give the same answer; the
    line reports both total query times, and per snapshot the performance
    ratio m_vis / (m n_active) and its inverse (n_active = nodes with an
    edge)."""
    import numpy as np
    import torch
    from paper_1507_01490_amd import synth
    torch.cuda.set_device(0)
    t0 = time.time()
    snaps = synth.collaboration_snapshots(500_000, 125_000, 2.1, 200, 4, 16)
    log(f"[snapshots] generated {len(snaps)} snapshots in {time.time() - t0:.1f}s")
    k = 10
    rows, prev = [], None
    tot_cold = tot_warm = 0.0
    for t, g in enumerate(snaps):
        with bc.Graph(g.row_ptr, g.col) as G:
            kw = dict(mode="batched", width=256, defer_arcs=-1)  # the collaboration workload's knobs
            G.topk(k, **kw)  # warm-up: workspace and cached order
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            cold = G.topk(k, **kw)
            c1 = time.perf_counter()
            warm = G.topk(k, first=prev, **kw) if prev is not None else cold
            c2 = time.perf_counter()
        assert cold.ids.tolist() == warm.ids.tolist() and cold.farness.tolist() == warm.farness.tolist()
        n_act = int((np.diff(g.row_ptr) > 0).sum())
        ms_c, ms_w = (c1 - c0) * 1e3, ((c2 - c1) * 1e3 if prev is not None else (c1 - c0) * 1e3)
        tot_cold += ms_c
        tot_warm += ms_w
        ratio = cold.stats["m_vis"] / (float(g.m) * max(n_act, 1))
        rows.append(dict(t=t + 1, m=g.m, n_active=n_act, ms_cold=round(ms_c, 2), ms_warm=round(ms_w, 2),
                         m_vis_cold=cold.stats["m_vis"], m_vis_warm=warm.stats["m_vis"], ratio=ratio,
                         inverse_ratio=1.0 / ratio if ratio > 0 else None))
        log(f"[snapshots] t={t + 1} m={g.m} cold {ms_c:.1f} ms warm {ms_w:.1f} ms ratio {ratio:.3e}")
        prev = cold.ids
    print(json.dumps(dict(metric="top-k closeness over a growing graph on 1 MI355X (cold vs warm-started order)",
                          value=round(tot_warm, 2), unit="ms (16 snapshots, warm)", cold_ms=round(tot_cold, 2),
                          speedup=round(tot_cold / tot_warm, 3), higher_is_better=False, rows=rows,
                          data="synthetic", config=dict(workload="collaboration snapshots: 500,000 actors, "
                                                                 "125,000 groups, Zipf(2.1) sizes <= 200, seed 4, "
                                                                 "16 snapshots", k=k, mode="batched", width=256,
                                                      defer_arcs=-1))), flush=True)


def serve_bench(args, bc, workloads):
    """Serving mix: capacity from a closed-loop burst of every request, then
    an open loop with Poisson arrivals at `load` x capacity; latency of a
    request = finish - submit on the server's clock."""
    import numpy as np
    if args.lanes is None:
        args.lanes = 1 if args.queue else 4
    t0 = time.time()
    mix = workloads.serve_mix(count=args.mix_count, max_n=args.mix_max_n)
    log(f"[serve] generated {len(mix)} graphs (sum n = {sum(g.n for g, _ in mix)}, "
        f"sum arcs = {sum(g.m for g, _ in mix)}) in {time.time() - t0:.1f}s")
    if args.queue:
        # continuous batching: one running kernel drains a device-visible
        # queue; its node records (sized for the largest graph) take part of
        # the budget, so the budget is larger than for whole-request launches
        budget_mb = args.budget_mb if args.budget_mb != 2048 else 8192
        S = bc.Server(lanes=args.lanes, slots=args.serve_slots, budget_bytes=budget_mb << 20, queue=True,
                      queue_width=64, queue_slots=0)
    else:
        budget_mb = args.budget_mb
        S = bc.Server(lanes=args.lanes, slots=args.serve_slots, budget_bytes=budget_mb << 20)
    gids = [S.add_graph(g.row_ptr, g.col, directed=g.directed) for g, _ in mix]
    # per-request options by graph family (request i is family i % 3: ER, BA,
    # grid + shortcuts), as a client that knows its graphs would pass them:
    # grids have no hubs and deep searches, which 256-source batches of
    # nearby sources without deferral share best (3x on a 200k-node grid);
    # 32 workgroups keep such a request's working memory within the budget
    fam_opts = [dict(), dict(), dict(width=256, order="locality", defer_arcs=-1, slots=32)] if args.family_knobs \
        else [dict(), dict(), dict()]
    if args.queue and args.family_knobs:
        # the queue kernel has one width; the order is still per request
        fam_opts = [dict(), dict(), dict(order="locality")]

    def run(times):
        """Submit request i at times[i] seconds from now (None: all at once)."""
        tickets = []
        start = time.perf_counter()
        for i, (gid, (_, k)) in enumerate(zip(gids, mix)):
            if times is not None:
                delay = start + times[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets.append(S.submit(gid, k, mode="batched", **fam_opts[i % 3]))
        out = []
        for i, t in enumerate(tickets):
            wait_or_report(t, i)
            out.append(S.poll(t))
            if (i + 1) % 16 == 0:
                log(f"[serve] {i + 1}/{len(tickets)} done at {time.perf_counter() - start:.1f}s")
        return out, time.perf_counter() - start

    def wait_or_report(t, i):
        """Wait for a request; report the server's state every 20 s, and give
        up (an error, not a silent wait) after args.request_timeout seconds."""
        waited = 0
        while not S.wait(t, 20000):
            waited += 20
            log(f"[serve] request {i} still waiting after {waited} s; server {S.info()}")
            if waited >= args.request_timeout:
                raise RuntimeError(f"request {i} did not finish in {waited} s")

    for i, (gid, (g, _)) in enumerate(list(zip(gids, mix))[:8]):  # warm-up: library, kernels, pool
        t = S.submit(gid, 1, mode="batched")
        wait_or_report(t, i)
        S.poll(t)
        log(f"[serve] warm-up {i + 1}/8 (n={g.n}) done")
    burst, span = run(None)
    capacity = len(mix) / span
    log(f"[serve] burst: {len(mix)} requests in {span:.2f}s -> capacity {capacity:.1f} req/s")
    rate = args.load * capacity
    rng = np.random.Generator(np.random.PCG64(3))
    times = np.cumsum(rng.exponential(1.0 / rate, len(mix)))
    res, span2 = run(times)
    same = all(a.ids.tolist() == b.ids.tolist() and a.farness.tolist() == b.farness.tolist()
               for a, b in zip(burst, res))
    # visited arcs each request's searches scanned (GPU-counted m_vis; it
    # depends a little on when each threshold was published, so per run)
    mvis_burst = sum(int(r.stats["m_vis"]) for r in burst)
    mvis_open = sum(int(r.stats["m_vis"]) for r in res)
    lat = np.array([r.info["finish_ms"] - r.info["submit_ms"] for r in res])
    wait = np.array([r.info["start_ms"] - r.info["submit_ms"] for r in res])
    svc = np.array([r.info["finish_ms"] - r.info["start_ms"] for r in res])
    info = S.info()
    S.close()
    line = dict(metric="serving latency p50/p99 and throughput on 1 MI355X (512-graph top-k mix)",
                value=round(len(mix) / span2, 3), unit="req/s", n_gpus=1, higher_is_better=True,
                p50_ms=round(float(np.percentile(lat, 50)), 2), p99_ms=round(float(np.percentile(lat, 99)), 2),
                mean_ms=round(float(lat.mean()), 2), wait_p50_ms=round(float(np.percentile(wait, 50)), 2),
                wait_p99_ms=round(float(np.percentile(wait, 99)), 2),
                service_p50_ms=round(float(np.percentile(svc, 50)), 2),
                service_p99_ms=round(float(np.percentile(svc, 99)), 2),
                capacity_rps=round(capacity, 3), offered_rps=round(rate, 3), load=args.load,
                gteps_closed_loop=round(mvis_burst / span / 1e9, 2), gteps_open_loop=round(mvis_open / span2 / 1e9, 2),
                work_m_vis=dict(closed_loop=mvis_burst, open_loop=mvis_open,
                                kind="GPU-counted m_vis summed over the requests; the closed loop also uploads "
                                     "the graphs the warm-up did not"),
                same_results_burst_vs_poisson=bool(same), dtype="int64", data="synthetic",
                config=dict(workload=workloads.DESCRIPTION["serve512"] if args.mix_count == 512 and args.mix_max_n == 2e5
                            else f"serving mix: {args.mix_count} graphs n~logU[1e3,{args.mix_max_n:g}] (ER deg 8 / BA m=4 / "
                                 "grid+1% shortcuts), k~U{1,10,100}, seed=3", lanes=args.lanes,
                            slots=args.serve_slots, budget_mb=budget_mb, mode="batched",
                            queue=bool(args.queue), family_options=fam_opts),
                server=dict(uploads=info["uploads"], evictions=info["evictions"], peak_mb=round(info["peak_bytes"] / 2**20, 1),
                            completed=info["completed"], failed=info["failed"],
                            queue_launches=info["queue_launches"], queue_batches=info["queue_batches"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
