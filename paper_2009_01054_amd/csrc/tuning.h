// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, the stage-1 walks (F2 slices in LDS and their workgroups per
// launch, 16 bytes of rows per lane) and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   SLICE: ridge f64 x1; ridge f32 x1; batched f64 (64 problems, 8 RHS), per iteration
//          0: 0.1111, 0.0835, 9.0360  (score 1.208)
//          1: 0.0919, 0.0673, 7.6964  (score 1.000)
//   SLICEWGS: ridge f64 x1; ridge f32 x1
//        128: 0.1046, 0.0735  (score 1.136)
//        256: 0.0901, 0.0663  (score 1.002)
//        512: 0.0921, 0.0661  (score 1.011)
//   WIDE: ridge f64 x1; ridge f32 x1
//          0: 0.1178, 0.0845  (score 1.110)
//          1: 0.1026, 0.0787  (score 1.000)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1024, 0.0782  (score 1.000)
//          2: 0.1064, 0.0794  (score 1.027)
//          4: 0.1105, 0.0913  (score 1.122)
//   R1: ridge f64 x1; ridge f32 x1; batched f64 (64 problems, 8 RHS), per iteration
//          8: 0.1118, 0.1105, 7.6529  (score 1.273)
//         16: 0.0905, 0.0668, 7.6706  (score 1.004)
//         32: 0.0910, 0.0668, 7.6751  (score 1.005)
//         64: 0.0901, 0.0672, 7.6821  (score 1.004)
//        128: 0.0908, 0.0666, 7.6806  (score 1.004)
//   MAXR64: ridge f64 x8; batched f64 (64 problems, 8 RHS), per iteration
//          2: 0.7698, 7.6857  (score 1.047)
//          4: 0.7018, 8.6544  (score 1.061)
//          8: 1.7399, 13.6073  (score 2.095)
//   MAXR32: ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.4884, 5.2164  (score 1.396)
//          4: 0.3073, 4.2559  (score 1.000)
//          8: 0.5343, 5.1715  (score 1.454)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.7697, 0.5493, 7.4313  (score 1.462)
//          4: 0.7689, 0.4653, 5.6606  (score 1.263)
//          8: 0.7668, 0.3992, 4.7361  (score 1.130)
//         16: 0.7681, 0.3066, 4.3063  (score 1.003)
//         32: 0.7688, 0.3070, 4.2745  (score 1.001)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 16.0;
constexpr double kStage2TargetR8 = 32.0;
constexpr int kStage1KeysPerWave = 1;
constexpr int kStage1Wide = 1;
constexpr int kStage1Slice = 1;
constexpr int kStage1SliceWgs = 256;
constexpr int kMaxRhsBlockF64 = 2;
constexpr int kMaxRhsBlockF32 = 4;
// Dense-tile cost model: effective rates of the gather path (Theorem 1 flops
// per second, ridge workload) and of the matrix-core product M Vmat N^T
// (complete data, 4096 x 2048), and the output-tile count at which a GEMM
// keeps the matrix cores busy (from the ridge workload's shapes, 64 tiles).
constexpr double kGatherRateF64 = 9.97e+12;
constexpr double kGatherRateF32 = 1.37e+13;
constexpr double kTilesRateF64 = 4.5e+13;
constexpr double kTilesRateF32 = 1.01e+14;
constexpr double kTilesFull = 142.6;
// Batched CG with FP32 products: a problem whose active systems all have
// recurrence residuals below this level continues with FP64 products
// (GVT_F32_SWITCH overrides; 0 keeps FP32 products until certification).
// Measured on the 256-problem workload: switching at 1e-2, 1e-3 or 1e-4 took
// 6.39, 5.48 and 5.18 s against 4.97 s without, and converged 1532, 1537 and
// 1536 systems against 1536: the systems FP32 products miss are those FP64
// products converge only in the last 10% of the iteration cap.
constexpr double kF32SwitchRelres = 0.0;
}  // namespace gvt
