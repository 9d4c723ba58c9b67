// Stage-2 tile targets: outputs per F1 row per tile for each RHS class.
// Written by paper_2009_01054_amd/tune.py on AMD Radeon Graphics; measured times (ms):
//   class R1: ridge f64 x1; ridge f32 x1
//     target      8: 0.2050, 0.1526  (score 1.220)
//     target     16: 0.1767, 0.1193  (score 1.002)
//     target     32: 0.1769, 0.1190  (score 1.001)
//     target     64: 0.1765, 0.1197  (score 1.003)
//     target    128: 0.1774, 0.1190  (score 1.002)
//   class R8: ridge f64 x8; ridge f32 x8; batched f32 (64 problems, 8 RHS), per iteration
//     target      2: 2.0699, 0.8793, 8.4911  (score 1.150)
//     target      4: 2.0509, 0.7777, 7.2171  (score 1.042)
//     target      8: 1.9983, 0.7538, 6.9383  (score 1.009)
//     target     16: 2.0069, 0.7351, 7.0487  (score 1.008)
//     target     32: 2.0060, 0.7333, 7.1532  (score 1.012)
#pragma once

namespace gvt {
constexpr double kStage2TargetR1 = 32.0;
constexpr double kStage2TargetR8 = 16.0;
}  // namespace gvt
