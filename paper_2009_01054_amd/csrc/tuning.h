// Tuned launch shapes: stage-2 tile targets (outputs per group row per tile) for
// each RHS class, and the keys each wave walks in stage 1.
// Written by paper_2009_01054_amd/tune.py on gfx950; measured times (ms):
//   LDS: ridge f64 x1; ridge f32 x1
//          0: 0.1604, 0.0963  (score 1.000)
//          1: 0.2088, 0.1136  (score 1.239)
//   KPW: ridge f64 x1; ridge f32 x1
//          1: 0.1479, 0.0894  (score 1.002)
//          2: 0.1473, 0.0900  (score 1.003)
//          4: 0.1480, 0.0978  (score 1.048)
//   R1: ridge f64 x1; ridge f32 x1
//          8: 0.1803, 0.1262  (score 1.328)
//         16: 0.1454, 0.0892  (score 1.002)
//         32: 0.1446, 0.0898  (score 1.004)
//         64: 0.1448, 0.0894  (score 1.002)
//        128: 0.1458, 0.0899  (score 1.008)
//   MAXR: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 1.0566, 0.5943, 7.1096  (score 1.128)
//          4: 1.1038, 0.4755, 6.1912  (score 1.015)
//          8: 1.8292, 0.5896, 6.7899  (score 1.330)
//   R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//          2: 1.1928, 0.6734, 8.1585  (score 1.261)
//          4: 1.1614, 0.5266, 6.6703  (score 1.077)
//          8: 1.1185, 0.5296, 8.1834  (score 1.140)
//         16: 1.1263, 0.4825, 6.1314  (score 1.007)
//         32: 1.1099, 0.4802, 6.1842  (score 1.003)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 64.0;
constexpr double kStage2TargetR8 = 32.0;
constexpr int kStage1KeysPerWave = 1;
constexpr int kMaxRhsBlock = 4;
constexpr int kStage1LdsKeysPerWave = 4;
constexpr double kStage1LdsMinReuse = 1e300;  // LDS-staged stage 1 off
}  // namespace gvt
