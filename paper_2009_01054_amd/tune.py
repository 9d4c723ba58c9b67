"""Autotuner for the launch shapes of the two stages (run on the GPU).

Stage 2 cuts the (F1 row, S row) plane of a two-factor term into tiles of 32
group rows (F1 rows for blocks of 1-2 RHS, S rows for blocks of 4-8 RHS) by a
block of staged rows.  The block height is chosen at plan time from the
density of the outputs so that each group row of a tile holds about
``target`` outputs; a pass of the kernel serves a fixed number of outputs per
row and re-reads the staged rows, so the best target depends on how many
right-hand sides share a pass.  There is one target per RHS class.  Stage 1
walks key segments with one wave per key; the number of keys each wave walks
trades waves in flight against per-wave work.

Over a contiguous range of S rows a stage-1 lane can hold 16 bytes of
consecutive rows (one vector load per pair) instead of one row.
A product pass carries a block of up to 8 right-hand sides; larger blocks
reuse every gathered element more often but hold more accumulators per lane,
so the largest block a pass takes is tuned too, per product precision.

This script sweeps these knobs on synthetic workloads shaped like the
library's benchmarks, through the library's environment overrides
(GVT_STAGE1_WIDE, GVT_STAGE1_KPW, GVT_STAGE2_TARGET_R1, GVT_STAGE2_TARGET_R8,
GVT_MAX_RHS_BLOCK_F64, GVT_MAX_RHS_BLOCK_F32; all are read when a plan is built),
and writes the winners as a C++
header that ``build.py`` compiles into the library:

    python -m paper_2009_01054_amd.tune --out paper_2009_01054_amd/csrc/tuning.h

Score of a candidate: the geometric mean over the class's workloads of its
time divided by the best time of that workload.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

R1_CANDIDATES = (8.0, 16.0, 32.0, 64.0, 128.0)
R8_CANDIDATES = (2.0, 4.0, 8.0, 16.0, 32.0)
KPW_CANDIDATES = (1, 2, 4)
MAXR_CANDIDATES = (2, 4, 8)
WIDE_CANDIDATES = (0, 1)  # stage 1 over contiguous S rows: one row per lane, or 16 bytes of rows


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _events_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


_KNOBS = {0: "GVT_STAGE2_TARGET_R1", 1: "GVT_STAGE2_TARGET_R8", "kpw": "GVT_STAGE1_KPW",
          "wide": "GVT_STAGE1_WIDE", "maxr64": "GVT_MAX_RHS_BLOCK_F64", "maxr32": "GVT_MAX_RHS_BLOCK_F32"}


def _set_target(cls, value):
    os.environ[_KNOBS[cls]] = (str(int(value)) if cls in ("kpw", "wide", "maxr64", "maxr32")
                               else repr(float(value)))


def ridge_products(gvt, W, torch, nrhs, reps):
    """Workloads: products of the ridge workload (m=2000, q=500, n=200000), FP64 and FP32."""
    p = W.config2()
    dev = torch.device("cuda:0")
    D64 = torch.from_numpy(p["D"]).to(dev)
    T64 = torch.from_numpy(p["T"]).to(dev)
    c = torch.from_numpy(p["c"]).to(dev)
    e = torch.from_numpy(p["e"]).to(dev)
    n = len(p["c"])
    out = []
    for name, D, T in [("f64", D64, T64), ("f32", D64.float(), T64.float())]:
        V = torch.randn((nrhs, n), dtype=D.dtype, device=dev)
        U = torch.empty((1, nrhs, n), dtype=D.dtype, device=dev)

        def run(D=D, T=T, V=V, U=U):
            plan = gvt.gvt_plan_create("kronecker", D.shape, T.shape, (c, e), (c, e),
                                       flags=gvt.FLAG_SYMMETRIC_BASES)
            ms = _events_ms(torch, lambda: plan.execute(D, T, V.t(), out=U), reps)
            plan.close()
            return ms

        out.append((f"ridge {name} x{nrhs}", run))
    return out


def batched_iterations(gvt, W, torch, nprob, prec="f32"):
    """Workload: per-iteration time of the batched ridge solver (FP32 or FP64
    products) on the first `nprob` problems of the 256-problem set (difference
    of two capped solves)."""
    dev = torch.device("cuda:0")
    shapes = W.config5_shapes()[:nprob]
    probs = [W.config5_problem(i, sh) for i, sh in enumerate(shapes)]
    t = lambda x: torch.from_numpy(x).to(dev)  # noqa: E731
    dp = [dict(D=t(q["D"]), T=t(q["T"]), c=t(q["c"]), e=t(q["e"]), y=t(q["y"])) for q in probs]
    lams = list(W.LAMBDA_GRID)

    def solve(iters):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gvt.gvt_krr_cg_batched("kronecker", dp, lams, max_iter=iters, tol=1e-300,
                               matvec_prec=gvt.F32 if prec == "f32" else gvt.F64, check_every=4)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def run():
        solve(3)
        return (solve(19) - solve(3)) / 16 * 1e3

    return [(f"batched {prec} ({nprob} problems, 8 RHS), per iteration", run)]


def sweep(cls, candidates, workloads):
    table = {}
    for cand in candidates:
        _set_target(cls, cand)
        row = []
        for name, run in workloads:
            ms = run()
            row.append(ms)
            _log(f"[tune] {_KNOBS[cls]}={cand:g}: {name}: {ms:.4f} ms")
        table[cand] = row
    os.environ.pop(_KNOBS[cls], None)
    best_per = [min(table[c][k] for c in candidates) for k in range(len(workloads))]
    score = {c: math.exp(sum(math.log(table[c][k] / best_per[k]) for k in range(len(workloads)))
                         / len(workloads)) for c in candidates}
    winner = min(candidates, key=lambda c: score[c])
    return winner, table, score


def write_header(path, results, device):
    lines = ["// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for",
             "// each RHS class, and the keys each wave walks in stage 1.",
             "// Written by paper_2009_01054_amd/tune.py on " + device + "; measured times (ms):"]
    for key, (winner, table, score, names) in results.items():
        lines.append(f"//   {key}: " + "; ".join(names))
        for cand, row in table.items():
            lines.append(f"//     {cand:6g}: " + ", ".join(f"{x:.4f}" for x in row)
                         + f"  (score {score[cand]:.3f})")
    lines += ["#pragma once", "", "namespace gvt {",
              f"constexpr double kStage2TargetR1 = {results['R1'][0]:.1f};",
              f"constexpr double kStage2TargetR8 = {results['R8'][0]:.1f};",
              f"constexpr int kStage1KeysPerWave = {int(results['KPW'][0])};",
              f"constexpr int kStage1Wide = {int(results['WIDE'][0])};",
              f"constexpr int kMaxRhsBlockF64 = {int(results['MAXR64'][0])};",
              f"constexpr int kMaxRhsBlockF32 = {int(results['MAXR32'][0])};",
              "}  // namespace gvt", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc",
                                                  "tuning.h"))
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--batched-problems", type=int, default=64)
    args = ap.parse_args()

    import torch

    import paper_2009_01054_amd as gvt
    from paper_2009_01054_amd import workloads as W

    assert torch.cuda.is_available(), "the tuner measures on the GPU"
    gvt.load_library()
    device = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    r1 = ridge_products(gvt, W, torch, 1, args.reps)
    r8 = ridge_products(gvt, W, torch, 8, max(2, args.reps // 4)) + batched_iterations(
        gvt, W, torch, args.batched_problems)
    b64 = batched_iterations(gvt, W, torch, args.batched_problems, "f64")
    for _, run in r1:  # first launches (code loading, allocator growth) stay out of the sweeps
        run()
    results = {}
    # the class-0 target sets the tile height only where target / density is
    # below 64 rows, which the ridge products (density 0.2) never reach; the
    # batched FP64 solver's smaller, denser problems (blocks of 2 RHS) do
    for key, cls, cands, wl in (("WIDE", "wide", WIDE_CANDIDATES, r1),
                                ("KPW", "kpw", KPW_CANDIDATES, r1),
                                ("R1", 0, R1_CANDIDATES, r1 + b64),
                                ("MAXR64", "maxr64", MAXR_CANDIDATES, r8[:1] + b64),
                                ("MAXR32", "maxr32", MAXR_CANDIDATES, r8[1:]),
                                ("R8", 1, R8_CANDIDATES, r8)):
        winner, table, score = sweep(cls, cands, wl)
        results[key] = (winner, table, score, [n for n, _ in wl])
        if key.startswith("MAXR") or key == "WIDE":
            _set_target(cls, winner)  # the later sweeps run with the chosen walk and block caps
        _log(f"[tune] class {key}: target {winner:g}")
    write_header(args.out, results, device)
    print(f"wrote {args.out}: stage-1 keys per wave {results['KPW'][0]}, R1 target {results['R1'][0]:g}, "
          f"largest RHS block F64 {results['MAXR64'][0]} / F32 {results['MAXR32'][0]}, "
          f"R8 target {results['R8'][0]:g}")


if __name__ == "__main__":
    main()
