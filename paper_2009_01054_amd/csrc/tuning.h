// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1755, 0.1103  (score 1.008)
//          2: 0.1726, 0.1109  (score 1.003)
//          4: 0.1786, 0.1178  (score 1.051)
//   R1: ridge f64 x1; ridge f32 x1
//          8: 0.2041, 0.1522  (score 1.216)
//         16: 0.1788, 0.1189  (score 1.006)
//         32: 0.1785, 0.1183  (score 1.003)
//         64: 0.1775, 0.1196  (score 1.005)
//        128: 0.1786, 0.1188  (score 1.005)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 2.0586, 0.8747, 8.4489  (score 1.150)
//          4: 2.0303, 0.7808, 7.2601  (score 1.048)
//          8: 1.9597, 0.7463, 7.0419  (score 1.010)
//         16: 1.9658, 0.7253, 7.0319  (score 1.001)
//         32: 2.0023, 0.7387, 7.2150  (score 1.022)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 32.0;
constexpr double kStage2TargetR8 = 16.0;
constexpr int kStage1KeysPerWave = 2;
constexpr int kStage1LdsKeysPerWave = 4;
constexpr double kStage1LdsMinReuse = 1e300;  // LDS-staged stage 1 off
}  // namespace gvt
