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
consecutive rows (one vector load per pair) instead of one row, and where the
F2 columns' slices of a block of rows fit in LDS the walk can read them from
there (the slice walk), with a tuned number of workgroups per launch; the
wide-walk knobs are measured with the slice walk off, since that walk serves
the buffers the slice does not fit.
A product pass carries a block of up to 8 right-hand sides; larger blocks
reuse every gathered element more often but hold more accumulators per lane,
so the largest block a pass takes is tuned too, per product precision.

This script sweeps these knobs on synthetic workloads shaped like the
library's benchmarks, through the library's environment overrides
(GVT_STAGE1_SLICE, GVT_STAGE1_SLICE_WGS, GVT_STAGE1_WIDE, GVT_STAGE1_KPW,
GVT_STAGE2_TARGET_R1, GVT_STAGE2_TARGET_R8, GVT_MAX_RHS_BLOCK_F64,
GVT_MAX_RHS_BLOCK_F32; all are read when a plan is built),
measures the rates of the dense-tile cost model (gather path against matrix-core
products), and writes the winners and rates as a C++ header that ``build.py``
compiles into the library:

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
SLICE_CANDIDATES = (0, 1)  # stage 1 over F2 slices in LDS where they fit
SLICE_WGS_CANDIDATES = (128, 256, 512)  # workgroups of a slice-walk launch


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
          "wide": "GVT_STAGE1_WIDE", "maxr64": "GVT_MAX_RHS_BLOCK_F64", "maxr32": "GVT_MAX_RHS_BLOCK_F32",
          "slice": "GVT_STAGE1_SLICE", "slicewgs": "GVT_STAGE1_SLICE_WGS"}
_INT_KNOBS = ("kpw", "wide", "maxr64", "maxr32", "slice", "slicewgs")


def _set_target(cls, value):
    os.environ[_KNOBS[cls]] = (str(int(value)) if cls in _INT_KNOBS
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
    products) on the first `nprob` problems of the 256-problem set (median of
    three differences of two capped solves)."""
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
        # median of three differences: one slow short solve would otherwise
        # read as a fast iteration
        solve(3)
        d = sorted((solve(19) - solve(3)) / 16 * 1e3 for _ in range(3))
        return d[1]

    return [(f"batched {prec} ({nprob} problems, 8 RHS), per iteration", run)]


def cost_model(gvt, W, torch, reps):
    """Rates of the dense-tile cost model (tuning.h): the gather path's Theorem 1 flops per
    second on the ridge products; the matrix-core rate of the complete-data product on a
    4096 x 2048 grid; and the output-tile count at which a GEMM keeps the matrix cores busy,
    from the dense product of the ridge workload's shapes (2000 x 500 outputs, 64 tiles of
    128 x 128 per GEMM): rate(64 tiles) = full rate x 64 / kTilesFull."""
    dev = torch.device("cuda:0")
    p = W.config2()
    c, e = torch.from_numpy(p["c"]).to(dev), torch.from_numpy(p["e"]).to(dev)
    n = len(p["c"])
    rng = W.rng_for(4, 2)
    m, q = 4096, 2048
    Dm = torch.from_numpy(W.gaussian_kernel(rng.standard_normal((m, 32)))).to(dev)
    Tq = torch.from_numpy(W.gaussian_kernel(rng.standard_normal((q, 32)))).to(dev)
    Vm = torch.from_numpy(rng.standard_normal((m, q))).to(dev)
    Vr = torch.from_numpy(rng.standard_normal((2000, 500))).to(dev)
    out, tiles_full = {}, []
    for name, dt, pc in [("F64", torch.float64, gvt.F64), ("F32", torch.float32, gvt.F32)]:
        D, T = torch.from_numpy(p["D"]).to(dev, dt), torch.from_numpy(p["T"]).to(dev, dt)
        v = torch.randn(n, dtype=dt, device=dev)
        plan = gvt.gvt_plan_create("kronecker", D.shape, T.shape, (c, e), (c, e),
                                   flags=gvt.FLAG_SYMMETRIC_BASES | gvt.FLAG_NO_DENSE_TILES)
        cost = gvt.gvt_plan_info(plan)["cost_fma"]
        ms = _events_ms(torch, lambda: plan.execute(D, T, v), reps)
        plan.close()
        out[f"kGatherRate{name}"] = 2.0 * cost / (ms * 1e-3)
        Dd, Td, Vd = Dm.to(dt), Tq.to(dt), Vm.to(dt)
        ms = _events_ms(torch, lambda: gvt.gvt_dense_matvec(Dd, Td, Vd, prec=pc), max(2, reps // 4))
        full = 2.0 * (m * m * q + m * q * q) / (ms * 1e-3)
        out[f"kTilesRate{name}"] = full
        Vs = Vr.to(dt)
        ms = _events_ms(torch, lambda: gvt.gvt_dense_matvec(D, T, Vs, prec=pc), reps)
        small = 2.0 * (2000 * 2000 * 500 + 2000 * 500 * 500) / (ms * 1e-3)
        tiles_full.append(64.0 * full / small)
        _log(f"[tune] cost model {name}: gather {out[f'kGatherRate{name}'] / 1e12:.2f} TFLOP/s, "
             f"dense {full / 1e12:.1f} TFLOP/s, ridge-shape dense {small / 1e12:.1f} TFLOP/s")
    out["kTilesFull"] = max(64.0, math.sqrt(tiles_full[0] * tiles_full[1]))
    return out


# Not swept (a full batched solve per candidate): the residual level below which a
# batched FP32-product problem moves to FP64 products, with the measurement behind it.
F32_SWITCH = ("0.0", [
    "Batched CG with FP32 products: a problem whose active systems all have",
    "recurrence residuals below this level continues with FP64 products",
    "(GVT_F32_SWITCH overrides; 0 keeps FP32 products until certification).",
    "Measured on the 256-problem workload: switching at 1e-2, 1e-3 or 1e-4 took",
    "6.39, 5.48 and 5.18 s against 4.97 s without, and converged 1532, 1537 and",
    "1536 systems against 1536: the systems FP32 products miss are those FP64",
    "products converge only in the last 10% of the iteration cap."])


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


def write_header(path, results, device, rates):
    lines = ["// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for",
             "// each RHS class, the stage-1 walks (F2 slices in LDS and their workgroups per",
             "// launch, 16 bytes of rows per lane) and the keys each wave walks in stage 1.",
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
              f"constexpr int kStage1Slice = {int(results['SLICE'][0])};",
              f"constexpr int kStage1SliceWgs = {int(results['SLICEWGS'][0])};",
              f"constexpr int kMaxRhsBlockF64 = {int(results['MAXR64'][0])};",
              f"constexpr int kMaxRhsBlockF32 = {int(results['MAXR32'][0])};",
              "// Dense-tile cost model: effective rates of the gather path (Theorem 1 flops",
              "// per second, ridge workload) and of the matrix-core product M Vmat N^T",
              "// (complete data, 4096 x 2048), and the output-tile count at which a GEMM",
              "// keeps the matrix cores busy (from the ridge workload's shapes, 64 tiles).",
              f"constexpr double kGatherRateF64 = {rates['kGatherRateF64']:.3g};",
              f"constexpr double kGatherRateF32 = {rates['kGatherRateF32']:.3g};",
              f"constexpr double kTilesRateF64 = {rates['kTilesRateF64']:.3g};",
              f"constexpr double kTilesRateF32 = {rates['kTilesRateF32']:.3g};",
              f"constexpr double kTilesFull = {rates['kTilesFull']:.1f};"]
    lines += ["// " + t for t in F32_SWITCH[1]]
    lines += [f"constexpr double kF32SwitchRelres = {F32_SWITCH[0]};", "}  // namespace gvt", ""]
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
    # the slice walk first (on the ridge products and the batched FP64 solver, whose
    # smaller problems take it where their slices fit), then the wide walk's knobs
    # with the slice walk off: that walk serves the buffers the slice does not fit
    for key, cls, cands, wl in (("SLICE", "slice", SLICE_CANDIDATES, r1 + b64),
                                ("SLICEWGS", "slicewgs", SLICE_WGS_CANDIDATES, r1),
                                ("WIDE", "wide", WIDE_CANDIDATES, r1),
                                ("KPW", "kpw", KPW_CANDIDATES, r1),
                                ("R1", 0, R1_CANDIDATES, r1 + b64),
                                ("MAXR64", "maxr64", MAXR_CANDIDATES, r8[:1] + b64),
                                ("MAXR32", "maxr32", MAXR_CANDIDATES, r8[1:]),
                                ("R8", 1, R8_CANDIDATES, r8)):
        if key == "WIDE":
            _set_target("slice", 0)
        winner, table, score = sweep(cls, cands, wl)
        results[key] = (winner, table, score, [n for n, _ in wl])
        if key.startswith("MAXR") or key in ("WIDE", "SLICE", "SLICEWGS"):
            _set_target(cls, winner)  # the later sweeps run with the chosen walks and block caps
        if key == "KPW":
            _set_target("slice", results["SLICE"][0])
        _log(f"[tune] class {key}: target {winner:g}")
    rates = cost_model(gvt, W, torch, args.reps)
    write_header(args.out, results, device, rates)
    print(f"wrote {args.out}: stage-1 keys per wave {results['KPW'][0]}, R1 target {results['R1'][0]:g}, "
          f"largest RHS block F64 {results['MAXR64'][0]} / F32 {results['MAXR32'][0]}, "
          f"R8 target {results['R8'][0]:g}")


if __name__ == "__main__":
    main()
