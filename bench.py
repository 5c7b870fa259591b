"""Benchmark: CI tests/s and skeleton wall time of the reverse-order PC
skeleton on one MI355X.

Workload: linear-Gaussian SEM on an Erdos-Renyi DAG, p = 1000 variables,
expected degree 4, n = 10000 samples in FP32, alpha = 0.01, levels after
the first capped at max_level = 5.  One step = one whole skeleton call
(correlation matrix, the l = p-2 level, levels 5..0 with deletion) on data
already resident in HBM.  The headline form is the mixed one (bf16x3
correlation on MFMA, FP32 tests, FP64 re-run near the threshold); the
plain FP64 form and the learned form (mixed, candidates ordered by the
ranking MLP trained on scale-free graphs) are timed in the same run, and
the learned form is also timed against the mixed one on a held-out
scale-free workload (BA DAG, p = 1000, n = 10000, max_level = 3).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "er_p1000_n10000_d4"
SEED = 0
BA_WORKLOAD = "ba_p1000_n10000_m2"
BA_SEED = 2000  # a held-out seed of the ranker's evaluation set
FP32_PEAK_TFLOPS = 157.3   # MI355X published vector FP32
# HBM bytes per launch of the dominant kernel (triple_kernel<float, 2>, level
# 5 of the workload above) from the FETCH_SIZE and WRITE_SIZE counter runs in
# profiles/triple_kernel_er_p1000_n10000_d4.md, scaled by the copy-kernel
# calibration (fetch x2.000, write x1.000).  Valid only for the kernel source
# and launch table they were taken with: any change to either makes the
# figure null until the counters are taken again.
MEASURED_TRAFFIC = {"bytes_per_launch": 10110728.0,
                    "sha256": {"paper_2109_04626_amd/csrc/citest.hip":
                               "25b8ca328450813494936bfbe841142e20cf2a652dccc728506c3791b58be89b",
                               "paper_2109_04626_amd/tuning_gfx950.json":
                               "9b5ee9cd8fc56c7307853a22b4732f84004d394956b92179119b5f35944c27e9"}}


def measured_traffic():
    import hashlib

    for rel, want in MEASURED_TRAFFIC["sha256"].items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
        except OSError:
            return None
    return MEASURED_TRAFFIC["bytes_per_launch"]
FP64_PEAK_TFLOPS = 78.6    # MI355X published vector FP64


def flops_per_test(l: int) -> float:
    """Algorithmic flops of one test at level l, F(l) = l^3/3 + 2 l^2 + 6 l
    + 20: the Cholesky of the l x l block, the two triangular solves, the
    three dot products of H and the final scaling."""
    return l ** 3 / 3.0 + 2.0 * l * l + 6.0 * l + 20.0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def bytes_per_test(l: int, elem: int) -> float:
    """Algorithmic bytes: the distinct correlation entries one test reads
    (upper triangle of C_KK, C_Ki, C_Kj, C_ij)."""
    return elem * (l * l + 5 * l + 2) / 2.0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=1e9, help="oracle tests in the CPU sample (about 10 s on 16 cores)")
    ap.add_argument("--max-level", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-instance workload")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--profile-mixed", action="store_true",
                    help="profiling mode: only the mixed form on the headline workload, one short line")
    ap.add_argument("--profile-batch", choices=("host", "graph"), default=None,
                    help="profiling mode: only the 80-instance batch, host-driven or as one device graph")
    ap.add_argument("--copy-probe", action="store_true",
                    help="profiling mode: a plain device copy of 1 GiB, five times (HBM counter calibration)")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the context block (mixed-form variants, forward schedule, held-out scale-free seeds)")
    ap.add_argument("--eval-seeds", type=int, default=20, help="held-out scale-free seeds in the context block")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2109_04626_amd as fpc
    import semdata

    if args.copy_probe:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": dt * 1e3,
                          "GB_per_s": 2 * nbytes / dt / 1e9}), flush=True)
        return 0

    if args.profile_batch:
        base, boots, datas, cfg5 = semdata.batched_workload()
        base_d = torch.from_numpy(base).cuda()
        inst = [(base_d, torch.from_numpy(r).cuda()) for r in boots] + \
               [(torch.from_numpy(d).cuda(), None) for d in datas]
        ctx = fpc.Context(0)
        flags = fpc.FPC_FLAG_GRAPH if args.profile_batch == "graph" else 0
        for _ in range(args.warmup):
            fpc.fpc_skeleton_batch(ctx, inst, alpha=cfg5["alpha"], max_level=cfg5["max_level"],
                                   precision=fpc.FPC_PREC_MIXED, flags=flags)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs = fpc.fpc_skeleton_batch(ctx, inst, alpha=cfg5["alpha"], max_level=cfg5["max_level"],
                                          precision=fpc.FPC_PREC_MIXED, flags=flags)
        torch.cuda.synchronize()
        print(json.dumps({"form": f"batch-{args.profile_batch}", "instances": len(inst),
                          "ms_per_call": (time.perf_counter() - t0) / args.steps * 1e3,
                          "ran_as_graph": all(o["corr_ms"] == 0.0 for o in outs)}), flush=True)
        ctx.close()
        return 0

    over = {} if args.max_level is None else {"max_level": args.max_level}
    X, sem, cfg = semdata.workload(WORKLOAD, SEED, **over)
    Xd = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()
    ctx = fpc.Context(0)

    from paper_2109_04626_amd.learned import DEFAULT_MODEL

    model = fpc.fpc_mlp_init(ctx, np.load(DEFAULT_MODEL))

    def timed(X_dev, c, prec, m=None, **kw):
        def run():
            return fpc.fpc_skeleton(ctx, X_dev, alpha=c["alpha"], max_level=c["max_level"], precision=prec,
                                    order_model=m, **kw)

        for _ in range(args.warmup):
            run()
        # the results kept alive here make Python's cyclic collector pause
        # for tens of ms at random calls: it runs before, not inside, the
        # timed region
        gc.collect()
        gc.disable()
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs = []
            for _ in range(args.steps):
                outs.append(run())
                outs[-1]["wall_ms"] = (time.perf_counter() - t0) * 1e3
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            gc.enable()
        return dt, outs

    # plain = FP64 tests, lexicographic order; mixed = bf16x6 C + FP32 tests
    # with FP64 recheck; learned = mixed with the MLP-ranked candidate order
    if args.profile_mixed:
        dt, outs = timed(Xd, cfg, fpc.FPC_PREC_MIXED)
        lv5 = [x for x in outs[-1]["levels"] if x["level"] == cfg["max_level"]]
        print(json.dumps({"form": "mixed", "ms_per_step": dt / args.steps * 1e3,
                          "levels": [{k: x[k] for k in ("level", "tests_executed", "test_kernel_ms", "test_launches")}
                                     for x in lv5]}), flush=True)
        ctx.close()
        return 0
    forms = {"mixed": (fpc.FPC_PREC_MIXED, None), "plain": (fpc.FPC_PREC_FP64, None),
             "learned": (fpc.FPC_PREC_MIXED, model)}
    results = {}
    for name, (prec, m) in forms.items():
        results[name] = timed(Xd, cfg, prec, m)
        print(f"[bench] {name}: {results[name][0] / args.steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    # the learned order on the scale-free workload it was trained for
    Xb, _, cfg_b = semdata.workload(BA_WORKLOAD, BA_SEED)
    Xbd = torch.from_numpy(Xb).cuda()
    ba = {name: timed(Xbd, cfg_b, fpc.FPC_PREC_MIXED, m) for name, m in (("mixed", None), ("learned", model))}
    del Xbd
    # many instances in one call: 64 bootstrap resamples of one data set and
    # 16 data sets of uneven p, against the same instances one call each
    batched = None
    if not args.no_batched:
        base, boots, datas, cfg5 = semdata.batched_workload()
        base_d = torch.from_numpy(base).cuda()
        inst = [(base_d, torch.from_numpy(r).cuda()) for r in boots] + \
               [(torch.from_numpy(d).cuda(), None) for d in datas]

        def run_batch(flags=0):
            return fpc.fpc_skeleton_batch(ctx, inst, alpha=cfg5["alpha"], max_level=cfg5["max_level"],
                                          precision=fpc.FPC_PREC_MIXED, flags=flags)

        def run_singles():
            return [fpc.fpc_skeleton(ctx, X if r is None else X[r.long()], alpha=cfg5["alpha"],
                                     max_level=cfg5["max_level"], precision=fpc.FPC_PREC_MIXED) for X, r in inst]

        run_batch()
        gc.collect()
        gc.disable()
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.batch_steps):
                outs_b = run_batch()
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) / args.batch_steps
            # the whole call as one device graph (captured and launched once per call)
            run_batch(fpc.FPC_FLAG_GRAPH)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.batch_steps):
                outs_g = run_batch(fpc.FPC_FLAG_GRAPH)
            torch.cuda.synchronize()
            tg = (time.perf_counter() - t0) / args.batch_steps
            run_singles()
            gc.collect()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs_s = run_singles()
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
        finally:
            gc.enable()
        diff_b = [k for k, (a, b) in enumerate(zip(outs_b, outs_s)) if not np.array_equal(a["adj"], b["adj"])]
        diff_g = [k for k, (a, b) in enumerate(zip(outs_g, outs_b))
                  if not (np.array_equal(a["adj"], b["adj"]) and a["sepsets"] == b["sepsets"])]
        graph_ok = all(o["corr_ms"] == 0.0 for o in outs_g)  # graph mode reports no per-phase split
        same_b = not diff_b
        if diff_b:
            k = diff_b[0]
            print(f"[bench] batched: instances {diff_b} differ from one call each; instance {k} levels (level, "
                  f"deleted, rechecked): batch {[(x['level'], x['deleted'], x['tests_rechecked']) for x in outs_b[k]['levels']]} "
                  f"single {[(x['level'], x['deleted'], x['tests_rechecked']) for x in outs_s[k]['levels']]}",
                  file=sys.stderr, flush=True)
        tests_b = sum(o["total_tests"] for o in outs_b)
        req_b = sum(o["total_required"] for o in outs_b)
        batched = {"workload": f"64 bootstrap resamples of an ER p={cfg5['base_p']} deg={cfg5['degree']} data set "
                               f"+ 16 ER data sets p~U[{cfg5['p_lo']},{cfg5['p_hi']}], n={cfg5['n']} X f32, "
                               f"alpha={cfg5['alpha']}, max_level={cfg5['max_level']}, mixed",
                   "instances": len(inst), "ms_per_call": tb * 1e3, "one_call_each_ms": ts * 1e3,
                   "speedup_vs_one_call_each": ts / tb, "tests_per_call": tests_b,
                   "ci_tests_per_s": tests_b / tb, "tests_required_per_call": req_b,
                   "required_tests_per_s": req_b / tb, "skeletons_equal": same_b, "instances_differing": diff_b,
                   "graph_mode": {"ms_per_call": tg * 1e3, "speedup_vs_host_driven": tb / tg,
                                  "speedup_vs_one_call_each": ts / tg, "ran_as_graph": graph_ok,
                                  "equal_to_host_driven": not diff_g, "instances_differing": diff_g}}
        print(f"[bench] batched: {tb * 1e3:.1f} ms/call host-driven, {tg * 1e3:.1f} ms/call as one graph, "
              f"{ts * 1e3:.1f} ms one call each", file=sys.stderr,
              flush=True)
        del inst, base_d

    # context: the mixed form's trades, the forward schedule (Algorithm 1)
    # against the reverse one, and the learned order on held-out seeds
    context = None
    if not args.no_context:
        context = {}
        for name, kw in (("strict_z", dict(ill_cond_tau=-1.0)), ("c32_bf16x3", dict(c32_method=fpc.FPC_CORR_BF16X3)),
                         ("c32_fp32_of_fp64", dict(c32_method=fpc.FPC_CORR_FP32))):
            t, o = timed(Xd, cfg, fpc.FPC_PREC_MIXED, **kw)
            lvo = [x for x in o[-1]["levels"] if x["level"] != cfg["p"] - 2]
            context[name] = {"ms_per_step": t / args.steps * 1e3, "rechecked": sum(x["tests_rechecked"] for x in lvo),
                             "level_kernel_ms": sum(x["kernel_ms"] for x in lvo), "corr_ms": o[-1]["corr_ms"],
                             "corr_max_abs_err": o[-1]["corr_max_abs_err"],
                             "skeleton_equal": bool(np.array_equal(o[-1]["adj"], results["plain"][1][-1]["adj"]))}
            print(f"[bench] {name}: {context[name]['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
        # the same step as a batch of one in graph mode: every level's
        # candidate sets, tests and deletions on the device, one launch
        one = [(Xd, None)]
        kwg = dict(alpha=cfg["alpha"], max_level=cfg["max_level"], precision=fpc.FPC_PREC_MIXED,
                   flags=fpc.FPC_FLAG_GRAPH)
        fpc.fpc_skeleton_batch(ctx, one, **kwg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            og = fpc.fpc_skeleton_batch(ctx, one, **kwg)[0]
        torch.cuda.synchronize()
        ref = results["mixed"][1][-1]
        context["step_as_one_graph"] = {
            "ms_per_step": (time.perf_counter() - t0) / args.steps * 1e3, "ran_as_graph": og["corr_ms"] == 0.0,
            "equal_to_mixed": bool(np.array_equal(og["adj"], ref["adj"]) and og["sepsets"] == ref["sepsets"])}
        print(f"[bench] step as one graph: {context['step_as_one_graph']['ms_per_step']:.2f} ms/step", file=sys.stderr,
              flush=True)
        fwd = {}
        for wname, seed, prec in (("er_p20_n1000_d3", 0, fpc.FPC_PREC_FP64), ("paper_p95_n10000", 0, fpc.FPC_PREC_FP64),
                                  (WORKLOAD, SEED, fpc.FPC_PREC_MIXED)):
            Xw, _, cw = semdata.workload(wname, seed)
            Xwd = torch.from_numpy(Xw).cuda()
            row = {}
            for sname, sch, lev in (("reverse", fpc.FPC_REVERSE, cw["max_level"]), ("forward", fpc.FPC_FORWARD, -1)):
                o = fpc.fpc_skeleton(ctx, Xwd, alpha=cw["alpha"], max_level=lev, precision=prec, schedule=sch)
                t0 = time.perf_counter()
                o = fpc.fpc_skeleton(ctx, Xwd, alpha=cw["alpha"], max_level=lev, precision=prec, schedule=sch)
                row[sname] = {"tests_required": o["total_required"], "tests_executed": o["total_tests"],
                              "ms": (time.perf_counter() - t0) * 1e3, "edges": int(o["adj"].sum()) // 2,
                              "max_level": lev}
                row[sname + "_adj"] = o["adj"]
            a, b = row.pop("reverse_adj"), row.pop("forward_adj")
            row["edges_in_both"] = int((a & b).sum()) // 2
            row["reverse_vs_forward_required"] = row["forward"]["tests_required"] / max(row["reverse"]["tests_required"], 1)
            fwd[f"{wname} seed {seed}"] = row
            del Xwd
        context["forward_vs_reverse"] = fwd
        from paper_2109_04626_amd import learned

        ev = learned.evaluate(ctx, model, list(learned.EVAL_SEEDS)[: args.eval_seeds], verbose=False)
        context["learned_heldout"] = {
            "workload": f"{BA_WORKLOAD}, held-out seeds {ev['rows'][0]['seed']}..{ev['rows'][-1]['seed']}",
            "seeds": len(ev["rows"]), "tests_lex": ev["tests_lex"], "tests_learned": ev["tests_learned"],
            "ms_lex_total": ev["ms_lex"], "ms_learned_total": ev["ms_learned"],
            "ms_lex_mean": ev["ms_lex"] / len(ev["rows"]), "ms_learned_mean": ev["ms_learned"] / len(ev["rows"]),
            "learned_faster_seeds": sum(r["ms_learned"] < r["ms_lex"] for r in ev["rows"]),
            "all_same_skeleton": ev["all_same"]}
        print(f"[bench] held-out BA: lex {context['learned_heldout']['ms_lex_mean']:.2f} ms, learned "
              f"{context['learned_heldout']['ms_learned_mean']:.2f} ms", file=sys.stderr, flush=True)

    dt, outs = results["mixed"]
    last = outs[-1]
    ref_adj = results["plain"][1][-1]["adj"]
    same = bool(np.array_equal(last["adj"], ref_adj))
    same_learned = bool(np.array_equal(results["learned"][1][-1]["adj"], ref_adj))
    tests = sum(o["total_tests"] for o in outs)
    value = tests / dt

    # dominant kernel: the test kernel of the level with the most tests;
    # achieved = its algorithmic flops / the device time of its launches (HIP
    # events around each launch, on the stream it is launched on; the size
    # classes of a window run on two streams, so the time is the union of the
    # launch intervals, and avg_launch_ms that union over the launch count)
    lv = [x for x in last["levels"] if x["level"] != cfg["p"] - 2]
    kms = sum(x["kernel_ms"] for x in lv)
    dom = max(lv, key=lambda x: x["tests_executed"])
    dom_flops = dom["tests_executed"] * flops_per_test(dom["level"])
    achieved = dom_flops / (dom["test_kernel_ms"] / 1e3) / 1e12 if dom["test_kernel_ms"] > 0 else 0.0
    if args.verbose:
        for name, (_, o) in [("ba-mixed", ba["mixed"]), ("ba-learned", ba["learned"])]:
            w = np.diff([0.0] + [x["wall_ms"] for x in o])
            print(f"[bench] {name} per call wall: " + " ".join(f"{v:.2f}" for v in w), file=sys.stderr)
            print(f"[bench] {name} per call lib:  " + " ".join(f"{x['total_ms']:.2f}" for x in o), file=sys.stderr)
        for name in forms:
            o = results[name][1][-1]
            print(f"[bench] {name}: total_ms(lib)={o['total_ms']:.2f} corr={o['corr_ms']:.2f} "
                  f"first={o['first_level_ms']:.2f}", file=sys.stderr)
            for x in o["levels"]:
                print(f"   l={x['level']:4d} E={x['edges_eligible']:7d} maxm={x['max_cand']:4d} "
                      f"poss={x['tests_possible']:12d} exec={x['tests_executed']:12d} "
                      f"rechk={x['tests_rechecked']:8d} del={x['deleted']:7d} "
                      f"dev={x['kernel_ms']:8.3f} test={x['test_kernel_ms']:8.3f}/{x['test_launches']} "
                      f"level={x['level_ms']:8.3f}", file=sys.stderr)
    plain_last = results["plain"][1][-1]
    lvp = [x for x in plain_last["levels"] if x["level"] != cfg["p"] - 2]
    kms_p = sum(x["kernel_ms"] for x in lvp)

    line = {
        "metric": "CI tests/sec + skeleton wall time at p=1000,n=1e4; learned/mixed vs plain GPU",
        "value": value,
        "unit": "CI tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 tests + f64 recheck, bf16x6 C",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD} seed {SEED}: ER DAG p={cfg['p']} deg={cfg['degree']}, "
                               f"n={cfg['n']} X {cfg['x_dtype']}, alpha={cfg['alpha']}, "
                               f"max_level={cfg['max_level']}",
                   "form": "mixed"},
        "plain_ms_per_step": results["plain"][0] / args.steps * 1e3,
        "mixed_vs_plain_speedup": results["plain"][0] / dt,
        "learned_ms_per_step": results["learned"][0] / args.steps * 1e3,
        "learned_vs_plain_speedup": results["plain"][0] / results["learned"][0],
        "learned_vs_mixed_speedup": dt / results["learned"][0],
        "tests_per_step_learned": results["learned"][1][-1]["total_tests"],
        "skeleton_equal_mixed_plain": same,
        "skeleton_equal_learned_plain": same_learned,
        "scale_free": {"workload": f"{BA_WORKLOAD} seed {BA_SEED}: BA DAG m=2 p={cfg_b['p']}, n={cfg_b['n']}, "
                                   f"alpha={cfg_b['alpha']}, max_level={cfg_b['max_level']}",
                       "mixed_ms_per_step": ba["mixed"][0] / args.steps * 1e3,
                       "learned_ms_per_step": ba["learned"][0] / args.steps * 1e3,
                       "mixed_lib_ms_median": float(np.median([o["total_ms"] for o in ba["mixed"][1]])),
                       "learned_lib_ms_median": float(np.median([o["total_ms"] for o in ba["learned"][1]])),
                       "mixed_lib_ms_max": float(np.max([o["total_ms"] for o in ba["mixed"][1]])),
                       "tests_mixed": ba["mixed"][1][-1]["total_tests"],
                       "tests_learned": ba["learned"][1][-1]["total_tests"],
                       "skeleton_equal": bool(np.array_equal(ba["mixed"][1][-1]["adj"],
                                                             ba["learned"][1][-1]["adj"]))},
        "batched": batched,
        "tests_per_step": outs[-1]["total_tests"],
        "tests_required_per_step": outs[-1]["total_required"],
        "required_tests_per_s": outs[-1]["total_required"] * args.steps / dt,
        "edges": int(last["adj"].sum()) // 2,
        "level_kernel_ms_mixed": kms,
        "level_kernel_ms_plain": kms_p,
        "ci_tests_per_s_kernel": sum(x["tests_executed"] for x in lv) / (kms / 1e3) if kms else None,
        "corr_ms": last["corr_ms"],
        "first_level_ms": last["first_level_ms"],
        "corr_max_abs_err": last["corr_max_abs_err"],
        "rechecked": sum(x["tests_rechecked"] for x in lv),
        "dominant_kernel": {"level": dom["level"], "launches": dom["test_launches"],
                            "avg_launch_ms": dom["test_kernel_ms"] / max(dom["test_launches"], 1),
                            "tests": dom["tests_executed"], "flops_per_test": flops_per_test(dom["level"])},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic()},
        "context": context,
    }

    if not args.no_cpu_baseline:
        import oracle

        t0 = time.perf_counter()
        C = oracle.corr(X.astype(np.float64))
        res = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"], max_level=cfg["max_level"],
                              max_tests=int(args.cpu_budget), partial_ok=True)
        tc = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
        # one thread: the first level of the same workload, and the whole small workload
        p = cfg["p"]
        t0 = time.perf_counter()
        r1 = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"], max_level=cfg["max_level"], nthreads=1,
                             max_tests=p * (p - 1) // 2, partial_ok=True)
        t1 = time.perf_counter() - t0
        Xs, _, cs = semdata.workload("er_p20_n1000_d3", 0)
        t0 = time.perf_counter()
        rs = oracle.skeleton(oracle.corr(Xs), cs["n"], alpha=cs["alpha"], max_level=cs["max_level"], nthreads=1)
        ts = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": res["total_tests"] / tc, "unit": "CI tests/s",
                                "cores": threads, "kind": "oracle",
                                "sample": f"same workload: correlation + first level + the first "
                                          f"{res['total_tests']} tests (budget {int(args.cpu_budget)}), "
                                          f"{tc:.1f} s, FP64, OpenMP over edges",
                                "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
                                "one_thread": {"first_level": {"workload": WORKLOAD, "tests": int(r1["levels"][0][2]),
                                                               "s": float(r1["level_seconds"][0]),
                                                               "tests_per_s": int(r1["levels"][0][2]) /
                                                               float(r1["level_seconds"][0])},
                                               "er_p20_n1000_d3": {"tests": rs["total_tests"], "s": ts,
                                                                   "tests_per_s": rs["total_tests"] / ts}}}
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
