// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   LDS: ridge f64 x1; ridge f32 x1
//          0: 0.1234, 0.0863  (score 1.000)
//          1: 0.1857, 0.1080  (score 1.372)
//   WIDE: ridge f64 x1; ridge f32 x1
//          0: 0.1308, 0.0890  (score 1.109)
//          1: 0.1153, 0.0820  (score 1.000)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1139, 0.0811  (score 1.000)
//          2: 0.1170, 0.0821  (score 1.020)
//          4: 0.1194, 0.0958  (score 1.113)
//   R1: ridge f64 x1; ridge f32 x1
//          8: 0.1321, 0.1189  (score 1.322)
//         16: 0.1137, 0.0810  (score 1.013)
//         32: 0.1134, 0.0813  (score 1.013)
//         64: 0.1123, 0.0810  (score 1.006)
//        128: 0.1123, 0.0801  (score 1.000)
//   MAXR64: ridge f64 x8; batched f64 (64 problems, 8 RHS), per iteration
//          2: 0.8539, 12.1869  (score 1.010)
//          4: 1.0600, 11.9544  (score 1.114)
//          8: 1.7510, 16.1165  (score 1.663)
//   MAXR32: ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.6126, 9.3197  (score 1.358)
//          4: 0.4995, 6.1947  (score 1.000)
//          8: 0.5837, 6.8196  (score 1.134)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 0.9196, 0.6984, 8.1135  (score 1.244)
//          4: 0.9154, 0.5480, 6.7489  (score 1.077)
//          8: 0.9180, 0.5335, 6.0530  (score 1.031)
//         16: 0.9234, 0.4905, 6.1530  (score 1.010)
//         32: 0.9268, 0.4886, 6.1764  (score 1.011)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 128.0;
constexpr double kStage2TargetR8 = 16.0;
constexpr int kStage1KeysPerWave = 1;
constexpr int kStage1Wide = 1;
constexpr int kMaxRhsBlockF64 = 2;
constexpr int kMaxRhsBlockF32 = 4;
constexpr int kStage1LdsKeysPerWave = 4;
constexpr double kStage1LdsMinReuse = 1e300;  // LDS-staged stage 1 off
}  // namespace gvt
