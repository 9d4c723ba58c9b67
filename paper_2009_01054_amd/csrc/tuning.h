// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   WIDE: ridge f64 x1; ridge f32 x1
//          0: 0.1264, 0.0897  (score 1.129)
//          1: 0.1091, 0.0815  (score 1.000)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1079, 0.0815  (score 1.000)
//          2: 0.1099, 0.0851  (score 1.031)
//          4: 0.1137, 0.0939  (score 1.102)
//   R1: ridge f64 x1; ridge f32 x1; batched f64 (64 problems, 8 RHS), per iteration
//          8: 0.1257, 0.1211, 9.0697  (score 1.162)
//         16: 0.1158, 0.0859, 8.9787  (score 1.005)
//         32: 0.1162, 0.0869, 9.0060  (score 1.011)
//         64: 0.1148, 0.0858, 11.3898  (score 1.084)
//        128: 0.1142, 0.0864, 9.0310  (score 1.005)
//   MAXR64: ridge f64 x8; batched f64 (64 problems, 8 RHS), per iteration
//          2: 0.8625, 9.0377  (score 1.000)
//          4: 1.0308, 11.3215  (score 1.224)
//          8: 1.7661, 14.2640  (score 1.798)
//   MAXR32: ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.5783, 5.6837  (score 1.178)
//          4: 0.4749, 4.9903  (score 1.000)
//          8: 0.5802, 5.6796  (score 1.179)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.8699, 0.6954, 6.7380  (score 1.269)
//          4: 0.8610, 0.5280, 5.4298  (score 1.074)
//          8: 0.8705, 0.5492, 4.8566  (score 1.052)
//         16: 0.8599, 0.4813, 5.1444  (score 1.022)
//         32: 0.8686, 0.4776, 4.9891  (score 1.012)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 128.0;
constexpr double kStage2TargetR8 = 32.0;
constexpr int kStage1KeysPerWave = 1;
constexpr int kStage1Wide = 1;
constexpr int kMaxRhsBlockF64 = 2;
constexpr int kMaxRhsBlockF32 = 4;
// Dense-tile cost model (a plan of one Kronecker term): effective rates of the
// gather path (Theorem 1 flops per second, ridge workload) and of the
// matrix-core GEMMs of M Vmat N^T (complete-data workload, 8192 x 4096), and
// the output-tile count at which a GEMM keeps the matrix cores busy (the
// ridge workload's 2000 x 500 GEMMs, 64 tiles, ran at 1/6 of the full rate).
constexpr double kGatherRateF64 = 9.3e12;
constexpr double kGatherRateF32 = 11.6e12;
constexpr double kTilesRateF64 = 56.0e12;
constexpr double kTilesRateF32 = 118.0e12;
constexpr double kTilesFull = 384.0;
// Batched CG with FP32 products: a problem whose active systems all have
// recurrence residuals below this level continues with FP64 products
// (GVT_F32_SWITCH overrides; 0 keeps FP32 products until certification).
// Measured on the 256-problem workload: switching at 1e-2, 1e-3 or 1e-4 took
// 6.39, 5.48 and 5.18 s against 4.97 s without, and converged 1532, 1537 and
// 1536 systems against 1536: the systems FP32 products miss are those FP64
// products converge only in the last 10% of the iteration cap.
constexpr double kF32SwitchRelres = 0.0;
}  // namespace gvt
