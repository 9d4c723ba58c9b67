// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   WIDE: ridge f64 x1; ridge f32 x1
//          0: 0.1287, 0.0912  (score 1.118)
//          1: 0.1121, 0.0838  (score 1.000)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1098, 0.0837  (score 1.004)
//          2: 0.1117, 0.0830  (score 1.009)
//          4: 0.1148, 0.0933  (score 1.084)
//   R1: ridge f64 x1; ridge f32 x1; batched f64 (64 problems, 8 RHS), per iteration
//          8: 0.1271, 0.1213, 9.0141  (score 1.221)
//         16: 0.1059, 0.0802, 9.0393  (score 1.001)
//         32: 0.1068, 0.0803, 9.0507  (score 1.005)
//         64: 0.1059, 0.0802, 9.0557  (score 1.002)
//        128: 0.1068, 0.0801, 9.0480  (score 1.004)
//   MAXR64: ridge f64 x8; batched f64 (64 problems, 8 RHS), per iteration
//          2: 0.7881, 9.0392  (score 1.000)
//          4: 0.9883, 11.5277  (score 1.265)
//          8: 1.6924, 14.4786  (score 1.855)
//   MAXR32: ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.5567, 5.7363  (score 1.182)
//          4: 0.4514, 5.0667  (score 1.000)
//          8: 0.5503, 5.8510  (score 1.187)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.7943, 0.6553, 6.9319  (score 1.275)
//          4: 0.7873, 0.4926, 5.5461  (score 1.073)
//          8: 0.7885, 0.5108, 4.9480  (score 1.047)
//         16: 0.7902, 0.4490, 5.0690  (score 1.011)
//         32: 0.7852, 0.4476, 5.0768  (score 1.009)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 16.0;
constexpr double kStage2TargetR8 = 32.0;
constexpr int kStage1KeysPerWave = 1;
constexpr int kStage1Wide = 1;
constexpr int kMaxRhsBlockF64 = 2;
constexpr int kMaxRhsBlockF32 = 4;
// Dense-tile cost model: effective rates of the gather path (Theorem 1 flops
// per second, ridge workload) and of the matrix-core product M Vmat N^T
// (complete data, 4096 x 2048), and the output-tile count at which a GEMM
// keeps the matrix cores busy (from the ridge workload's shapes, 64 tiles).
constexpr double kGatherRateF64 = 8.45e+12;
constexpr double kGatherRateF32 = 1.15e+13;
constexpr double kTilesRateF64 = 4.46e+13;
constexpr double kTilesRateF32 = 1.03e+14;
constexpr double kTilesFull = 131.3;
// Batched CG with FP32 products: a problem whose active systems all have
// recurrence residuals below this level continues with FP64 products
// (GVT_F32_SWITCH overrides; 0 keeps FP32 products until certification).
// Measured on the 256-problem workload: switching at 1e-2, 1e-3 or 1e-4 took
// 6.39, 5.48 and 5.18 s against 4.97 s without, and converged 1532, 1537 and
// 1536 systems against 1536: the systems FP32 products miss are those FP64
// products converge only in the last 10% of the iteration cap.
constexpr double kF32SwitchRelres = 0.0;
}  // namespace gvt
