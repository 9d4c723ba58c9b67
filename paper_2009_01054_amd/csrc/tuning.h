// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   LDS: ridge f64 x1; ridge f32 x1
//          0: 0.1406, 0.0932  (score 1.000)
//          1: 0.1855, 0.1087  (score 1.241)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1326, 0.0903  (score 1.000)
//          2: 0.1338, 0.0911  (score 1.009)
//          4: 0.1370, 0.0992  (score 1.066)
//   R1: ridge f64 x1; ridge f32 x1
//          8: 0.1470, 0.1255  (score 1.295)
//         16: 0.1288, 0.0881  (score 1.015)
//         32: 0.1280, 0.0872  (score 1.007)
//         64: 0.1278, 0.0871  (score 1.006)
//        128: 0.1273, 0.0865  (score 1.000)
//   MAXR64: ridge f64 x8; batched f64 (64 problems, 8 RHS), per iteration
//          2: 0.8954, 12.2322  (score 1.016)
//          4: 1.0977, 11.8597  (score 1.107)
//          8: 1.8186, 16.2070  (score 1.666)
//   MAXR32: ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.6320, 9.5217  (score 1.433)
//          4: 0.4744, 6.1803  (score 1.000)
//          8: 0.5878, 6.6582  (score 1.155)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.9743, 0.6738, 8.0772  (score 1.240)
//          4: 0.9744, 0.5265, 6.7524  (score 1.076)
//          8: 0.9818, 0.5225, 6.0088  (score 1.035)
//         16: 0.9797, 0.4777, 6.2174  (score 1.016)
//         32: 0.9794, 0.4745, 6.1962  (score 1.012)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 128.0;
constexpr double kStage2TargetR8 = 32.0;
constexpr int kStage1KeysPerWave = 1;
constexpr int kMaxRhsBlockF64 = 2;
constexpr int kMaxRhsBlockF32 = 4;
constexpr int kStage1LdsKeysPerWave = 4;
constexpr double kStage1LdsMinReuse = 1e300;  // LDS-staged stage 1 off
}  // namespace gvt
