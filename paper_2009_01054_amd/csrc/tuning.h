// Stage-2 tile targets: outputs per F1 row per tile for each RHS class.
// Written by paper_2009_01054_amd/tune.py on AMD Radeon Graphics; measured times (ms):
//   class R1: ridge f64 x1; ridge f32 x1
//     target      8: 0.2078, 0.1530  (score 1.215)
//     target     16: 0.1802, 0.1198  (score 1.001)
//     target     32: 0.1813, 0.1200  (score 1.005)
//     target     64: 0.1803, 0.1204  (score 1.004)
//     target    128: 0.1799, 0.1199  (score 1.001)
//   class R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//     target      2: 1.9060, 0.7062, 7.3493  (score 1.000)
//     target      4: 2.0142, 0.7842, 7.4009  (score 1.057)
//     target      8: 2.2084, 0.8065, 7.5592  (score 1.108)
//     target     16: 2.9579, 1.0107, 7.6324  (score 1.321)
//     target     32: 2.9472, 1.0098, 7.9277  (score 1.336)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 128.0;
constexpr double kStage2TargetR8 = 2.0;
}  // namespace gvt
