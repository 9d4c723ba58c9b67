// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, the stage-1 walks (F2 slices in LDS and their workgroups per
// launch, 16 bytes of rows per lane) and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   SLICE: ridge f64 x1; ridge f32 x1; batched f64 (64 problems, 8 RHS), per iteration
//          0: 0.1126, 0.0847, 9.0405  (score 1.228)
//          1: 0.0896, 0.0679, 7.6560  (score 1.000)
//   SLICEWGS: ridge f64 x1; ridge f32 x1
//        128: 0.1024, 0.0725  (score 1.127)
//        256: 0.0885, 0.0663  (score 1.002)
//        512: 0.0909, 0.0660  (score 1.014)
//   WIDE: ridge f64 x1; ridge f32 x1
//          0: 0.1159, 0.0841  (score 1.106)
//          1: 0.1018, 0.0783  (score 1.000)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1012, 0.0782  (score 1.000)
//          2: 0.1043, 0.0790  (score 1.021)
//          4: 0.1093, 0.0924  (score 1.130)
//   R1: ridge f64 x1; ridge f32 x1; batched f64 (64 problems, 8 RHS), per iteration
//          8: 0.1095, 0.1150, 7.6473  (score 1.292)
//         16: 0.0903, 0.0663, 7.6420  (score 1.009)
//         32: 0.0892, 0.0664, 7.6991  (score 1.007)
//         64: 0.0887, 0.0659, 7.6905  (score 1.002)
//        128: 0.0890, 0.0666, 7.6941  (score 1.007)
//   MAXR64: ridge f64 x8; batched f64 (64 problems, 8 RHS), per iteration
//          2: 0.7641, 7.6564  (score 1.000)
//          4: 1.0073, 9.2551  (score 1.262)
//          8: 1.6973, 13.6275  (score 1.988)
//   MAXR32: ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.5030, 5.2170  (score 1.152)
//          4: 0.4014, 4.9257  (score 1.000)
//          8: 0.5300, 5.6682  (score 1.233)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.7634, 0.6074, 6.7219  (score 1.295)
//          4: 0.7671, 0.4399, 5.4001  (score 1.083)
//          8: 0.7576, 0.4654, 4.7869  (score 1.055)
//         16: 0.7683, 0.3960, 4.9243  (score 1.014)
//         32: 0.7588, 0.3979, 4.8987  (score 1.010)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 64.0;
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
constexpr double kGatherRateF32 = 1.34e+13;
constexpr double kTilesRateF64 = 4.32e+13;
constexpr double kTilesRateF32 = 1.04e+14;
constexpr double kTilesFull = 150.9;
// Batched CG with FP32 products: a problem whose active systems all have
// recurrence residuals below this level continues with FP64 products
// (GVT_F32_SWITCH overrides; 0 keeps FP32 products until certification).
// Measured on the 256-problem workload: switching at 1e-2, 1e-3 or 1e-4 took
// 6.39, 5.48 and 5.18 s against 4.97 s without, and converged 1532, 1537 and
// 1536 systems against 1536: the systems FP32 products miss are those FP64
// products converge only in the last 10% of the iteration cap.
constexpr double kF32SwitchRelres = 0.0;
}  // namespace gvt
