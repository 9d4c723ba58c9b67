// Gather-path kernels of the generalized vec trick (Theorem 1) for gfx950.
//
// One Kronecker term u_i = sum_j F1[x_i, k_j] F2[y_i, o_j] v_j is applied in
// two stages:
//   stage 1 (segmented scatter-reduce):  S[y, k] = sum_{j: k_j = k} F2[y, o_j] v_j
//   stage 2 (gather-dot):                u_i    = sum_k F1[x_i, k] S[y_i, k]
// Input pairs are pre-sorted by the key k into contiguous segments, so every
// sum is a sequential loop or a fixed lane tree: results are deterministic
// (no atomics).  Several right-hand sides (R) ride along in the innermost
// dimension so that each gathered base-matrix element feeds R FMAs.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "tuning.h"

namespace gvt {

static constexpr int WAVE = 64;

__device__ __forceinline__ int wave_id_uniform() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <class T> struct Vec16;  // 16-byte vector of T
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };

// ---------------------------------------------------------------------------
// vs[p*R + r] = V[perm[p] + r*ldv]  (input vector gathered into key order)
template <class T>
__global__ void pack_v_kernel(const T *__restrict__ V, int64_t ldv, const int32_t *__restrict__ perm,
                              int64_t n, int R, T *__restrict__ vs, const int *__restrict__ gate) {
  if (gate && *gate == 0) return;
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t j = perm[p];
  for (int r = 0; r < R; ++r) vs[p * R + r] = V[j + r * ldv];
}

// s[k*R + r] = sum_{p in seg(k)} vs[p*R + r]   (segment sums, sequential per key)
template <class T>
__global__ void segsum_kernel(const int64_t *__restrict__ seg, const T *__restrict__ vs,
                              int64_t nkeys, int R, T *__restrict__ s) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  int64_t p0 = seg[k], p1 = seg[k + 1];
  for (int r = 0; r < R; ++r) {
    T acc = T(0);
    for (int64_t p = p0; p < p1; ++p) acc += vs[p * R + r];
    s[k * R + r] = acc;
  }
}

// ---------------------------------------------------------------------------
// Stage 1 (segmented scatter-reduce).  Fc holds F2 column-accessible:
// F2[y, o] = Fc[o*ldc + y].  Block = 4 waves over 64 S rows (one per lane);
// each wave owns KPW consecutive keys and walks each key's segment: the
// pair's other index and packed v value are wave-uniform scalar loads, the
// column load is coalesced over the 64 rows, and the loop is unrolled so
// that several column loads are in flight.  Pairs inside a segment are
// ordered by other index, which keeps consecutive column loads close in the
// cache.  The [64 x KB*R] result tile is staged in LDS and written
// row-contiguously.
// One wave instruction copying 64 x 16 bytes from global memory into LDS:
// lane i reads 16 bytes at its own address g and they land at bytes 16i..16i+15
// after l (l must be the same for the whole wave).
__device__ __forceinline__ void lds_load_row16(const void *g, void *l) {
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 16, 0, 0);
}

template <class T, int R, int KPW_ = 4> struct S1Cfg {
  static constexpr int KPW = KPW_;     // keys per wave
  static constexpr int KB = 4 * KPW;   // keys per block
};

// Body of one stage-1 block (key block kb, row block rb); shared by the
// single-product kernel and the grouped kernel of batched products.
template <class T, int R, int KPW = 4>
__device__ __forceinline__ void stage1_block(const T *__restrict__ Fc, int64_t ldc,
                                             const int32_t *__restrict__ rows, int64_t nrows,
                                             const int64_t *__restrict__ seg,
                                             const int32_t *__restrict__ other,
                                             const T *__restrict__ vs, int64_t nkeys,
                                             T *__restrict__ S, int64_t ldS, int64_t kb, int64_t rb,
                                             T *stg) {
  typedef S1Cfg<T, R, KPW> C;
  constexpr int W = C::KB * R;
  const int lane = threadIdx.x & 63;
  const int w = wave_id_uniform();
  const int64_t k0 = kb * C::KB;
  const int64_t rho0 = rb * 64;
  const int64_t rho = rho0 + lane;
  const bool live = rho < nrows;
  const int64_t y = live ? rows[rho] : 0;
#pragma unroll 1
  for (int kk = 0; kk < C::KPW; ++kk) {
    const int64_t k = k0 + w * C::KPW + kk;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
    if (k < nkeys) {
      const int64_t p0 = seg[k], p1 = seg[k + 1];
      const T *fy = Fc + y;
#pragma unroll 8
      for (int64_t p = p0; p < p1; ++p) {
        const T f = fy[(int64_t)other[p] * ldc];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += f * vs[p * R + r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) stg[lane * (W + 1) + (w * C::KPW + kk) * R + r] = acc[r];
  }
  __syncthreads();
  const int64_t kcount = (nkeys - k0) < C::KB ? (nkeys - k0) : C::KB;
  const int width = (int)kcount * R;
  for (int idx = threadIdx.x; idx < 64 * W; idx += 256) {
    const int rr = idx / W, cc = idx - rr * W;
    const int64_t orow = rho0 + rr;
    if (orow < nrows && cc < width) S[orow * ldS + k0 * R + cc] = stg[rr * (W + 1) + cc];
  }
  // the last key block also clears the row padding (read by stage 2 as whole chunks)
  if (k0 + C::KB >= nkeys) {
    const int64_t padw = ldS - nkeys * R;
    for (int64_t idx = threadIdx.x; idx < 64 * padw; idx += 256) {
      const int64_t rr = idx / padw, cc = idx - rr * padw;
      if (rho0 + rr < nrows) S[(rho0 + rr) * ldS + nkeys * R + cc] = T(0);
    }
  }
}

template <class T, int R, int KPW>
__global__ __launch_bounds__(256) void stage1_kernel(
    const T *__restrict__ Fc, int64_t ldc, const int32_t *__restrict__ rows, int64_t nrows,
    const int64_t *__restrict__ seg, const int32_t *__restrict__ other, const T *__restrict__ vs,
    int64_t nkeys, T *__restrict__ S, int64_t ldS, const int *__restrict__ gate) {
  __shared__ T stg[64 * (S1Cfg<T, R, KPW>::KB * R + 1)];
  if (gate && *gate == 0) return;
  stage1_block<T, R, KPW>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, blockIdx.x, blockIdx.y,
                          stg);
}

// Stage 1 over a contiguous range of S rows (S row i is F2 row row0 + i), each
// lane holding VPL = 16 / sizeof(T) consecutive rows: one 16-byte load per pair
// and lane fetches the lane's rows of the F2 column, so a block covers 64 * VPL
// rows with the load instructions of 64.  The loads need only T's own
// alignment (the hardware serves dword-aligned 16-byte global loads).  The lane
// that straddles the end of the range loads the range's last VPL rows and keeps
// the ones that are its own, so no load leaves the range (nrows >= VPL).  Each
// (row, key) sum runs over the key's segment in the same order as in the
// one-row walk, so the two agree bit for bit.
template <class T> struct Vec16u;  // 16 bytes of T at T's alignment
template <> struct Vec16u<double> { typedef double type __attribute__((ext_vector_type(2), aligned(8))); };
template <> struct Vec16u<float> { typedef float type __attribute__((ext_vector_type(4), aligned(4))); };

template <class T, int R, int KPW> struct S1WideCfg {
  static constexpr int VPL = 16 / sizeof(T);  // rows per lane
  static constexpr int ROWS = 64 * VPL;       // rows per block
  static constexpr int KB = 4 * KPW;          // keys per block
  static constexpr int W = KB * R;            // staged columns
  static constexpr int STG = ROWS * (W + 1);  // staged elements
};

template <class T, int R, int KPW>
__device__ __forceinline__ void stage1_wide_block(const T *__restrict__ Fc, int64_t ldc, int64_t row0,
                                                  int64_t nrows, const int64_t *__restrict__ seg,
                                                  const int32_t *__restrict__ other,
                                                  const T *__restrict__ vs, int64_t nkeys,
                                                  T *__restrict__ S, int64_t ldS, int64_t kb, int64_t rb,
                                                  T *stg) {
  typedef S1WideCfg<T, R, KPW> C;
  typedef typename Vec16u<T>::type V;
  constexpr int VPL = C::VPL, KB = C::KB, W = C::W, ROWS = C::ROWS;
  const int lane = threadIdx.x & 63;
  const int w = wave_id_uniform();
  const int64_t k0 = kb * KB;
  const int64_t rho0 = rb * ROWS;
  const int64_t rho = rho0 + lane * VPL;
  // the lane's rows, or the range's last VPL rows for the lane that straddles
  // its end (window rows before `shift` belong to the previous lane) and for
  // lanes past it (shift = VPL: they keep nothing)
  const int64_t base = rho + VPL <= nrows ? rho : nrows - VPL;
  const int shift = (int)(rho - base < VPL ? rho - base : VPL);
  const T *fy = Fc + row0 + base;
#pragma unroll 1
  for (int kk = 0; kk < KPW; ++kk) {
    const int64_t k = k0 + w * KPW + kk;
    T acc[R][VPL];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < VPL; ++j) acc[r][j] = T(0);
    if (k < nkeys) {
      const int64_t p0 = seg[k], p1 = seg[k + 1];
#pragma unroll 8
      for (int64_t p = p0; p < p1; ++p) {
        const V f = *reinterpret_cast<const V *>(fy + (int64_t)other[p] * ldc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T x = vs[p * R + r];
#pragma unroll
          for (int j = 0; j < VPL; ++j) acc[r][j] += f[j] * x;
        }
      }
    }
    T *st = stg + (w * KPW + kk) * R;
    if (shift == 0) {  // every lane but the one at the ragged end
#pragma unroll
      for (int j = 0; j < VPL; ++j)
#pragma unroll
        for (int r = 0; r < R; ++r) st[(lane * VPL + j) * (W + 1) + r] = acc[r][j];
    } else {
#pragma unroll
      for (int j = 0; j < VPL; ++j)
        if (j >= shift)
#pragma unroll
          for (int r = 0; r < R; ++r) st[(lane * VPL + j - shift) * (W + 1) + r] = acc[r][j];
    }
  }
  __syncthreads();
  const int64_t kcount = (nkeys - k0) < KB ? (nkeys - k0) : KB;
  const int width = (int)kcount * R;
  for (int idx = threadIdx.x; idx < ROWS * W; idx += 256) {
    const int rr = idx / W, cc = idx - rr * W;
    const int64_t orow = rho0 + rr;
    if (orow < nrows && cc < width) S[orow * ldS + k0 * R + cc] = stg[rr * (W + 1) + cc];
  }
  if (k0 + KB >= nkeys) {
    const int64_t padw = ldS - nkeys * R;
    for (int64_t idx = threadIdx.x; idx < ROWS * padw; idx += 256) {
      const int64_t rr = idx / padw, cc = idx - rr * padw;
      if (rho0 + rr < nrows) S[(rho0 + rr) * ldS + nkeys * R + cc] = T(0);
    }
  }
}

template <class T, int R, int KPW>
__global__ __launch_bounds__(256) void stage1_wide_kernel(
    const T *__restrict__ Fc, int64_t ldc, int64_t row0, int64_t nrows,
    const int64_t *__restrict__ seg, const int32_t *__restrict__ other, const T *__restrict__ vs,
    int64_t nkeys, T *__restrict__ S, int64_t ldS, int64_t nkb, int64_t per,
    const int *__restrict__ gate) {
  __shared__ T stg[S1WideCfg<T, R, KPW>::STG];
  if (gate && *gate == 0) return;
  // per == 0: a 2-D grid (key block, row block).  Otherwise, for F2 row sets
  // larger than an L2: workgroups go to the 8 XCDs in turn (workgroup i to
  // XCD i % 8), and block b of the (row block, key block) order, key blocks
  // fastest, runs as workgroup b % per of XCD b / per, so each XCD walks a
  // contiguous run of row blocks and their F2 rows stay in its L2 while all
  // key blocks read them.
  int64_t kb = blockIdx.x, rb = blockIdx.y;
  if (per > 0) {
    const int64_t b = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (b >= nkb * ((nrows + S1WideCfg<T, R, KPW>::ROWS - 1) / S1WideCfg<T, R, KPW>::ROWS)) return;
    kb = b % nkb;
    rb = b / nkb;
  }
  stage1_wide_block<T, R, KPW>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, S, ldS, kb, rb, stg);
}

// Degenerate stage 1 (key == other index): S[rho, k] = F2[rows[rho], k] * s[k].
template <class T>
__global__ void colscale_kernel(const T *__restrict__ F, int64_t ldf, const int32_t *__restrict__ rows,
                                int64_t nrows, const T *__restrict__ s, int64_t nkeys, int R,
                                T *__restrict__ S, int64_t ldS) {
  // one thread per (row, padded key slot); slots past nkeys are zero padding
  const int64_t kslots = ldS / R;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = nrows * kslots;
  if (idx >= total) return;
  int64_t rho = idx / kslots, k = idx - rho * kslots;
  if (k < nkeys) {
    T f = F[(int64_t)rows[rho] * ldf + k];
    for (int r = 0; r < R; ++r) S[rho * ldS + k * R + r] = f * s[k * R + r];
  } else {
    for (int r = 0; r < R; ++r) S[rho * ldS + k * R + r] = T(0);
  }
}

// ---------------------------------------------------------------------------
// Stage 2 (gather-dot), 2-D tiles.  The plan cuts the (x, S-row) plane into
// tiles of 32 consecutive F1 rows x one block of at most 64 S rows, orders
// the outputs by (tile, x, S row), and numbers the tiles so that the S-row
// block index is the fastest-varying digit.  Workgroups are dealt to the
// eight XCDs round-robin by id; the kernel remaps ids so that XCD x runs the
// F1 blocks x, x + 8, ..., each with all its S blocks in turn: an XCD reads
// one eighth of F1 once, and its tiles in flight walk the key chunks of all
// of S together, so S is shared through L2 (ridge workload, FP64: 100 MB
// fetched per launch against 266 MB when each XCD owned one S block and
// streamed all of F1, and 64 against 68-70 us).  S is then re-read once per
// F1 block, which the memory-side cache serves while F1 and S fit in it; past
// that the launch keeps the S-block order (fused four-kind FP64 product at
// m = 5000: 400 MB, stage 2 4.36 against 4.84 ms by F1 block).
// GVT_STAGE2_XCD=0 / 1 forces either order.
// Inside a tile one 16-lane group owns one F1 row: it holds that row's slice
// of the current key chunk in registers (loaded once per chunk) and walks
// its outputs, reading the S rows from a shared LDS tile (one 1 KB chunk per
// S row).  Partial sums stay in registers across chunks and meet in a fixed
// butterfly at the end, so the result is deterministic.
// Sum over the 16 lanes of a DPP row, in every lane, by data-parallel moves
// inside the row (quad swaps, then half-row and row mirrors): no LDS traffic.
// Each add pairs two partial sums, so every lane ends with the same value.
template <int CTRL> __device__ __forceinline__ int dpp_mov(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(dpp_mov<CTRL>(__float_as_int(x)));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_mov<CTRL>((int)(b & 0xffffffffll)), hi = dpp_mov<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <class T> __device__ __forceinline__ T row16_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_mov<0x141>(v);  // row_half_mirror: quad q <-> the mirrored quad of its half
  v += dpp_mov<0x140>(v);  // row_mirror: half <-> other half
  return v;
}

// Largest value of x over the wave (x per 16-lane group), as a scalar.
__device__ __forceinline__ int wave_max_of_groups(int x) {
  x = max(x, __shfl_xor(x, 16));
  x = max(x, __shfl_xor(x, 32));
  return __builtin_amdgcn_readfirstlane(x);
}

// Stage 1 with a slice of F2 resident in LDS.  A workgroup owns RB = 16 x VPL
// consecutive S rows, 256 bytes of each F2 column, and first copies those rows
// of every column into LDS (column o at byte 256 o); it then walks the
// segments of a range of keys.  Each 16-lane group of a wave walks one key, so
// a wave has four keys in flight: the group's lanes load the (other, v) of 16
// consecutive pairs, and at each step a DPP row broadcast hands every lane of
// the group that pair's column and v; the lane reads its VPL rows of the
// column with one 16-byte LDS read and accumulates.  Operand bytes come from
// LDS instead of through the vector-memory path, which bounds the walks that
// load a column slice per pair.  Each (row, key) sum runs over the segment in
// order, as in the other walks, so all of them agree bit for bit (steps past
// a segment's end add F2 x 0, which leaves a finite sum unchanged).  The last
// row block starts nrows - RB rows in, so no copy leaves the rows the buffer
// needs; its lanes keep only the rows past the previous block.
template <class T> struct S1SliceCfg {
  static constexpr int VPL = 16 / sizeof(T);  // rows per lane
  static constexpr int RB = 16 * VPL;         // rows per block: 256 bytes of a column
  static constexpr int NW = 16;               // waves per workgroup
  static constexpr int NT = 64 * NW;
};
// Largest number of F2 columns whose slices fit in LDS.
constexpr int64_t kS1SliceMaxCols = 600;

// value of lane s of this lane's 16-lane row (DPP row_newbcast)
template <int S> __device__ __forceinline__ int row_bcast(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x150 + S, 0xf, 0xf, false);
}
template <int S> __device__ __forceinline__ float row_bcast(float x) {
  return __int_as_float(row_bcast<S>(__float_as_int(x)));
}
// 64-bit values move in one DPP instruction (gfx90a and later allow row_newbcast on them)
template <int S> __device__ __forceinline__ long long row_bcast(long long x) {
  return __builtin_amdgcn_update_dpp(0LL, x, 0x150 + S, 0xf, 0xf, false);
}
template <int S> __device__ __forceinline__ double row_bcast(double x) {
  return __longlong_as_double(row_bcast<S>(__double_as_longlong(x)));
}

// Body of one slice-walk workgroup (key range kr of kpr keys, row block rb);
// shared by the single-product kernel and the grouped kernel of batched
// products.  s1s_lds: the dynamic LDS of at least nother x 256 bytes.
template <class T, int R>
__device__ __forceinline__ void stage1_slice_block(
    const T *__restrict__ Fc, int64_t ldc, int64_t row0, int64_t nrows,
    const int64_t *__restrict__ seg, const int32_t *__restrict__ other, const T *__restrict__ vs,
    int64_t nkeys, int64_t nother, T *__restrict__ S, int64_t ldS, int64_t kpr, int64_t kr, int64_t rb,
    unsigned char *s1s_lds) {
  typedef S1SliceCfg<T> C;
  typedef typename Vec16u<T>::type VG;  // 16 bytes at T's alignment (global)
  typedef typename Vec16<T>::type VL;   // 16-byte aligned (LDS)
  constexpr int VPL = C::VPL, RB = C::RB;
  constexpr bool kPackCV = sizeof(T) == 4 && R == 1;
  // Global address space spelled out: the pointers may come from a descriptor
  // in memory, and loads through flat pointers would also count against the
  // LDS wait counter, so every wait for a column read would wait for them too.
  typedef const __attribute__((address_space(1))) VG *GVG;
  const __attribute__((address_space(1))) T *Fg = (const __attribute__((address_space(1))) T *)Fc;
  const __attribute__((address_space(1))) int64_t *segg = (const __attribute__((address_space(1))) int64_t *)seg;
  const __attribute__((address_space(1))) int32_t *otherg =
      (const __attribute__((address_space(1))) int32_t *)other;
  const __attribute__((address_space(1))) T *vsg = (const __attribute__((address_space(1))) T *)vs;
  __attribute__((address_space(1))) T *Sg = (__attribute__((address_space(1))) T *)S;
  const int64_t rstart = rb * RB;                                      // first row stored
  const int64_t base = rstart + RB <= nrows ? rstart : nrows - RB;     // window inside [0, nrows)
  const int shift = (int)(rstart - base);                              // window rows before rstart
  {
    // piece q = 16 o + pc: 16 bytes of column o at byte 16 q; a thread's eight
    // pieces are loaded together, then stored
    const __attribute__((address_space(1))) T *src = Fg + row0 + base;
    const int64_t nvec = nother * 16;
    for (int64_t q0 = threadIdx.x; q0 < nvec; q0 += 8 * C::NT) {
      VL tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t q = q0 + (int64_t)u * C::NT;
        if (q < nvec) tmp[u] = *reinterpret_cast<GVG>(src + (q >> 4) * ldc + (q & 15) * VPL);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t q = q0 + (int64_t)u * C::NT;
        if (q < nvec) *reinterpret_cast<VL *>(s1s_lds + q * 16) = tmp[u];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, sub = lane & 15;
  const int sub16 = sub * 16;  // this lane's 16 bytes of a column slice
  const int wv = threadIdx.x >> 6;
  const int64_t k0 = kr * kpr;
  const int64_t k1 = k0 + kpr < nkeys ? k0 + kpr : nkeys;
  // segment bounds of the group's key, loaded one key quad ahead
  int64_t s0n = 0, s1n = 0;
  if (k0 + 4 * wv + g < k1) {
    s0n = segg[k0 + 4 * wv + g];
    s1n = segg[k0 + 4 * wv + g + 1];
  }
  for (int64_t kq = k0 + 4 * wv; kq < k1; kq += 4 * C::NW) {  // uniform
    const int64_t k = kq + g;
    const bool kv = k < k1;
    const int64_t s0 = s0n, s1 = s1n;
    if (kq + 4 * C::NW + g < k1) {
      s0n = segg[kq + 4 * C::NW + g];
      s1n = segg[kq + 4 * C::NW + g + 1];
    }
    const int maxlen = wave_max_of_groups((int)(s1 - s0));
    T acc[VPL][R];
#pragma unroll
    for (int j = 0; j < VPL; ++j)
#pragma unroll
      for (int r = 0; r < R; ++r) acc[j][r] = T(0);
    // the (other, v) of the group's next 16 pairs, loaded one window ahead
    int64_t pn = s0 + sub;
    bool inn = pn < s1;
    int coln = inn ? otherg[pn] * 256 : 0;  // byte offset of the pair's column slice
    T vln[R];
#pragma unroll
    for (int r = 0; r < R; ++r) vln[r] = inn ? vsg[pn * R + r] : T(0);
    for (int w0 = 0; w0 < maxlen; w0 += 16) {
      const int col = coln;
      T vl[R];
#pragma unroll
      for (int r = 0; r < R; ++r) vl[r] = vln[r];
      if (w0 + 16 < maxlen) {  // uniform
        pn += 16;
        inn = pn < s1;
        coln = inn ? otherg[pn] * 256 : 0;
#pragma unroll
        for (int r = 0; r < R; ++r) vln[r] = inn ? vsg[pn * R + r] : T(0);
      }
      const int nst = maxlen - w0;  // uniform
// the window's column reads are issued first (16 in flight, 8 with eight RHS), then the sums
// (FP32 with one RHS: the column offset and v move together in one 64-bit broadcast)
#define GVT_S1S_RD(SS)                                                                     \
  if constexpr (kPackCV) {                                                                 \
    const long long cv = row_bcast<SS>(colv);                                              \
    xv[SS] = __int_as_float((int)(cv >> 32));                                              \
    tv[SS] = *reinterpret_cast<const VL *>(s1s_lds + (int)(cv & 0xffffffffll) + sub16);    \
  } else {                                                                                 \
    tv[SS] = *reinterpret_cast<const VL *>(s1s_lds + row_bcast<SS>(col) + sub16);          \
  }
#define GVT_S1S_ACC(SS)                                                                    \
  _Pragma("unroll") for (int r = 0; r < R; ++r) {                                          \
    T x;                                                                                   \
    if constexpr (kPackCV) x = xv[SS];                                                     \
    else x = row_bcast<SS>(vl[r]);                                                         \
    _Pragma("unroll") for (int j = 0; j < VPL; ++j) acc[j][r] += tv[SS][j] * x;            \
  }
#define GVT_S1S_RD4(S4) GVT_S1S_RD(S4) GVT_S1S_RD(S4 + 1) GVT_S1S_RD(S4 + 2) GVT_S1S_RD(S4 + 3)
#define GVT_S1S_ACC4(S4) GVT_S1S_ACC(S4) GVT_S1S_ACC(S4 + 1) GVT_S1S_ACC(S4 + 2) GVT_S1S_ACC(S4 + 3)
      VL tv[16];
      [[maybe_unused]] T xv[16];
      [[maybe_unused]] long long colv = 0;
      if constexpr (kPackCV)
        colv = ((long long)__float_as_int((float)vl[0]) << 32) | (long long)(unsigned)col;
      if constexpr (R < 8) {
        if (nst > 8) {  // a whole window (or most of the last one)
          GVT_S1S_RD4(0) GVT_S1S_RD4(4) GVT_S1S_RD4(8) GVT_S1S_RD4(12)
          GVT_S1S_ACC4(0) GVT_S1S_ACC4(4) GVT_S1S_ACC4(8) GVT_S1S_ACC4(12)
        } else {  // the last window's first eight steps
          GVT_S1S_RD4(0) GVT_S1S_RD4(4)
          GVT_S1S_ACC4(0) GVT_S1S_ACC4(4)
        }
      } else {  // eight RHS: eight reads in flight (registers)
        GVT_S1S_RD4(0) GVT_S1S_RD4(4)
        GVT_S1S_ACC4(0) GVT_S1S_ACC4(4)
        if (nst > 8) {
          GVT_S1S_RD4(8) GVT_S1S_RD4(12)
          GVT_S1S_ACC4(8) GVT_S1S_ACC4(12)
        }
      }
#undef GVT_S1S_ACC4
#undef GVT_S1S_RD4
#undef GVT_S1S_ACC
#undef GVT_S1S_RD
    }
    if (kv) {
#pragma unroll
      for (int j = 0; j < VPL; ++j) {
        const int rr = sub * VPL + j;
        if (rr >= shift)
#pragma unroll
          for (int r = 0; r < R; ++r) Sg[(base + rr) * ldS + k * R + r] = acc[j][r];
      }
    }
  }
  // the last key range also clears the padding columns of the block's rows
  // (stage 2 reads S rows as whole chunks)
  if (k1 == nkeys) {
    const int64_t padw = ldS - nkeys * R;
    const int64_t nr = (nrows - rstart < RB ? nrows - rstart : RB);
    for (int64_t idx = threadIdx.x; idx < nr * padw; idx += C::NT) {
      const int64_t rr = idx / padw, cc = idx - rr * padw;
      Sg[(rstart + rr) * ldS + nkeys * R + cc] = T(0);
    }
  }
}

template <class T, int R>
__global__ __launch_bounds__(S1SliceCfg<T>::NT) void stage1_slice_kernel(
    const T *__restrict__ Fc, int64_t ldc, int64_t row0, int64_t nrows,
    const int64_t *__restrict__ seg, const int32_t *__restrict__ other, const T *__restrict__ vs,
    int64_t nkeys, int64_t nother, T *__restrict__ S, int64_t ldS, int64_t kpr,
    const int *__restrict__ gate) {
  extern __shared__ __attribute__((aligned(16))) unsigned char s1s_lds[];
  if (gate && *gate == 0) return;
  stage1_slice_block<T, R>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, kpr, blockIdx.x,
                           blockIdx.y, s1s_lds);
}

template <class T, int R> struct S2Cfg {
  static constexpr int LPO = 16;                   // lanes per F1 row / output
  static constexpr int NG = kStage2Rows;           // groups = F1 rows per tile (32)
  static constexpr int NT = NG * LPO;              // threads per workgroup (512)
  static constexpr int VEC = 16 / sizeof(T);       // elements per 16-byte LDS read
  static constexpr int EPL = VEC > R ? VEC : R;    // elements per lane per step
  static constexpr int KPL = EPL / R;              // keys per lane per step
  static constexpr int ROWE = 1024 / sizeof(T);    // tile row: 1 KB
  static constexpr int KC = ROWE / R;              // keys per chunk
  static constexpr int STEPS = KC / (LPO * KPL);
  // outputs per group per pass: 32 accumulators per lane, 64 for FP32 with
  // four or more RHS (fewer passes, each re-copying the S tile)
  static constexpr int ACC = (sizeof(T) == 4 && R >= 4) ? 64 : 32;
  static constexpr int OPG = (ACC / R) > 4 ? ACC / R : 4;
  // outputs per batch, whose S reads are in flight together; idle slots cost
  // reads too (measured on the ridge workload: FP64 one RHS 72 us with 4 against
  // 74 with 2 and 85 with 1; two RHS 149 us with 2 against 155 with 4; FP32 one
  // RHS 52 us with 2 against 53-54 with 4, two RHS 90 against 99)
  static constexpr int OB = (sizeof(T) == 8 && R == 1) ? 4 : 2;
  // tile row stride: 1 KB for FP64, 1 KB + 16 B for FP32 (measured on the
  // ridge workload: FP64 76 us unpadded against 92 us with 16 B, 82 us with
  // 128 B; FP32 52 us with 16 B against 62 us unpadded)
  static constexpr int PADE = sizeof(T) == 8 ? 0 : VEC;
  static_assert(STEPS >= 1, "chunk smaller than one step");
};

template <class T, int R> struct S2Smem {
  __attribute__((aligned(16))) T tile[kStage2MaxS * (S2Cfg<T, R>::ROWE + S2Cfg<T, R>::PADE)];
  __attribute__((aligned(4))) unsigned char meta[S2Cfg<T, R>::NG][S2Cfg<T, R>::OPG];
};

// Body of one stage-2 tile t; shared by the single-product kernel and the
// grouped kernel of batched products.
template <class T, int R>
__device__ __forceinline__ void stage2_tile(
    const T *__restrict__ F1, int64_t ld1, int64_t nx, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tiley, const int32_t *__restrict__ tilemax,
    const uint8_t *__restrict__ grow, const int32_t *__restrict__ yrows,
    const int32_t *__restrict__ perm, int nyb, const T *__restrict__ S, int64_t ldS, int64_t nkeys,
    T coef, T *__restrict__ out, int64_t ldi, int64_t ldr, int t, S2Smem<T, R> &sm) {
  typedef S2Cfg<T, R> C;
  typedef typename Vec16<T>::type V16;
  constexpr int TROW = C::ROWE + C::PADE;
  T *tile = sm.tile;
  auto &meta = sm.meta;
  const int maxcnt = tilemax[t];
  if (maxcnt == 0) return;  // uniform: empty tile
  const int xb = t / nyb;
  const int64_t y0 = tiley[2 * t], nyr = tiley[2 * t + 1];
  const int sub = threadIdx.x % C::LPO, grp = threadIdx.x / C::LPO;
  // the tile's rows by descending output count: a wave's four groups carry
  // similar counts, so few output slots run idle behind the wave's largest
  const int gr = grow[(int64_t)t * C::NG + grp];
  const int64_t x = (int64_t)xb * C::NG + gr;
  const int64_t qb = tileoff[(int64_t)t * (C::NG + 1) + gr];
  const int cnt = (int)(tileoff[(int64_t)t * (C::NG + 1) + gr + 1] - qb);
  const T *frow = F1 + (x < nx ? x : 0) * ld1;
  const int64_t nch = (nkeys + C::KC - 1) / C::KC;
  for (int pass0 = 0; pass0 < maxcnt; pass0 += C::OPG) {
    const int npass = (cnt - pass0) < C::OPG ? (cnt - pass0) : C::OPG;  // may be <= 0
    __syncthreads();
    for (int o = sub; o < C::OPG; o += C::LPO)
      meta[grp][o] = (o < npass) ? (unsigned char)(yrows[qb + pass0 + o] - y0) : 0;
    // FP32: this group's S-row bytes for the pass, packed four to a register
    // (FP64 has no registers to spare and reads them from LDS per chunk)
    constexpr bool kPack = sizeof(T) == 4;
    static_assert(C::OPG % 4 == 0, "whole 32-bit words of meta");
    unsigned mp[C::OPG / 4];
    if (kPack) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < C::OPG / 4; ++j) mp[j] = *reinterpret_cast<const unsigned *>(&meta[grp][4 * j]);
    }
    T acc[C::OPG][R];
#pragma unroll
    for (int o = 0; o < C::OPG; ++o)
#pragma unroll
      for (int r = 0; r < R; ++r) acc[o][r] = T(0);
    for (int64_t c = 0; c < nch; ++c) {
      __syncthreads();
      // S rows are padded with zeros to whole chunks, so every row is a full
      // 1 KB: one wave instruction moves a row from global memory straight into
      // its LDS tile row (lane i fills bytes 16i..16i+15), without registers,
      // and all of a wave's rows are in flight together
      {
        const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
        static_assert(C::ROWE * sizeof(T) == 64 * 16, "a tile row is one wave-wide 16-byte load");
        for (int row = wv; row < nyr; row += C::NT / 64)
          lds_load_row16(S + (y0 + row) * ldS + c * C::ROWE + ln * C::VEC, tile + row * TROW);
      }
      T dsl[C::STEPS][C::KPL];
      const int64_t k0 = c * C::KC;
#pragma unroll
      for (int st = 0; st < C::STEPS; ++st)
#pragma unroll
        for (int j = 0; j < C::KPL; ++j) {
          const int64_t kk = k0 + (int64_t)st * C::LPO * C::KPL + sub * C::KPL + j;
          dsl[st][j] = (npass > 0 && x < nx && kk < nkeys) ? frow[kk] : T(0);
        }
      __builtin_amdgcn_s_waitcnt(0);  // the tile rows have landed in LDS
      __syncthreads();
      // outputs in batches of OB behind one branch: slots past npass read tile
      // row 0 (meta is 0 there) into accumulators that are never stored, so the
      // reads of a batch's outputs are in flight together at every step
      static_assert(C::OPG % C::OB == 0, "whole batches of outputs");
#pragma unroll
      for (int o0 = 0; o0 < C::OPG; o0 += C::OB) {
        if (o0 < npass) {
          const T *trow[C::OB];
#pragma unroll
          for (int q = 0; q < C::OB; ++q) {
            const int o = o0 + q;
            const int mrow = kPack ? (int)((mp[o >> 2] >> (8 * (o & 3))) & 0xffu) : (int)meta[grp][o];
            trow[q] = tile + mrow * TROW + sub * C::EPL;
          }
#pragma unroll
          for (int st = 0; st < C::STEPS; ++st) {
            V16 sv[C::OB][C::EPL / C::VEC];
#pragma unroll
            for (int q = 0; q < C::OB; ++q)
#pragma unroll
              for (int u0 = 0; u0 < C::EPL / C::VEC; ++u0)
                sv[q][u0] = *reinterpret_cast<const V16 *>(trow[q] + st * C::LPO * C::EPL + u0 * C::VEC);
#pragma unroll
            for (int q = 0; q < C::OB; ++q)
#pragma unroll
              for (int u = 0; u < C::EPL; ++u)
                acc[o0 + q][u % R] += dsl[st][u / R] * sv[q][u / C::VEC][u % C::VEC];
          }
        }
      }
    }
    // lane partial sums meet inside each 16-lane row; slots past every
    // group's count in this wave are skipped (wave-uniform bound)
    static_assert(C::LPO == 16, "one DPP row per output");
    const int wn = wave_max_of_groups(npass);
#pragma unroll
    for (int o = 0; o < C::OPG; ++o) {
      if (o < wn) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[o][r] = row16_sum(acc[o][r]);
      }
      if (sub == 0 && o < npass) {
        const int64_t i = perm[qb + pass0 + o];
#pragma unroll
        for (int r = 0; r < R; ++r) out[i * ldi + r * ldr] = coef * acc[o][r];
      }
    }
  }
}

template <class T, int R>
__global__ __launch_bounds__(kStage2Rows * 16) void stage2_kernel(
    const T *__restrict__ F1, int64_t ld1, int64_t nx, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tiley, const int32_t *__restrict__ tilemax,
    const uint8_t *__restrict__ grow, const int32_t *__restrict__ yrows,
    const int32_t *__restrict__ perm, int nyb, const T *__restrict__ S, int64_t ldS, int64_t nkeys,
    T coef, T *__restrict__ out, int64_t ldi, int64_t ldr, const int *__restrict__ gate, int nxb,
    int by_f1) {
  __shared__ S2Smem<T, R> sm;
  if (gate && *gate == 0) return;
  int t = blockIdx.x;
  if (by_f1) {
    // workgroups go to the 8 XCDs round-robin by id: XCD x runs the F1 blocks
    // xb = x (mod 8), each with all its S blocks in turn (F1 blocks padded to a
    // multiple of 8; padding tiles return at once)
    const int x = t & 7, k = t >> 3;
    const int xb = (k / nyb) * 8 + x, yb = k % nyb;
    if (xb >= nxb) return;
    t = xb * nyb + yb;
  }
  stage2_tile<T, R>(F1, ld1, nx, tileoff, tiley, tilemax, grow, yrows, perm, nyb, S, ldS, nkeys, coef,
                    out, ldi, ldr, t, sm);
}

// ---------------------------------------------------------------------------
// Stage 2 at low output density (one RHS).  A workgroup takes a dual tile:
// 128 F1 rows x the S rows of two consecutive S-row blocks, the union of 4 x 2
// tiles of stage2_kernel (the same output order, perm and tile offsets).  Both
// operands are staged in LDS in chunks of 256 bytes of every row (128 F1 rows
// and up to 128 S rows, 64 KB per chunk, two buffers: the next chunk's rows are
// copied global-to-LDS while the current one is walked), so a staged row
// serves all of the tile's outputs in its row, about 5 at 4% density against
// 1.3 for an S row staged for 32 F1 rows.  The workgroup's 64 groups of 16
// lanes take its outputs in turn (output i to group i mod 64, at most 16 per
// group and pass); per chunk a group reads each output's two rows (one 16-byte
// LDS read each per lane) and accumulates in registers.  Each lane sums the
// same keys in the same order as in stage2_kernel (16 consecutive bytes of
// every 256), and the lanes meet in the same DPP row sum, so the two kernels
// give the same bits.  Dual tiles go to the XCDs in regions of 4 x 8 (512 F1
// rows, up to 1 024 S rows), so an XCD's 32 CUs walk rows that share its L2.
template <class T> struct S2dCfg {
  static constexpr int NG = 64, NT = NG * 16;  // 16-lane groups, threads
  static constexpr int SX = 4, SY = 2;         // stage2_kernel tiles per dual tile
  static constexpr int XT = SX * kStage2Rows;  // 128 F1 rows
  static constexpr int YT = SY * kStage2MaxS;  // at most 128 S rows
  static constexpr int CB = 256;               // bytes of a row per chunk
  static constexpr int KC = CB / (int)sizeof(T);
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int OPG = 16;               // outputs per group per pass
  static constexpr int NV = (XT + YT) * CB / 16;  // one chunk's rows in 16-byte units (64 KB)
  static constexpr int RX = 4, RY = 8;         // dual tiles per XCD region
};

template <class T>
__global__ __launch_bounds__(S2dCfg<T>::NT) void stage2_dual_kernel(
    const T *__restrict__ F1, int64_t ld1, int64_t nx, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tiley, int nxb, int nyb, const int32_t *__restrict__ yrows,
    const int32_t *__restrict__ perm, const T *__restrict__ S, int64_t ldS, int64_t nsrows, int64_t nkeys,
    T coef, T *__restrict__ out, int64_t ldi, const int *__restrict__ gate) {
  typedef S2dCfg<T> C;
  typedef typename Vec16<T>::type V;
  // the two chunk buffers are separate arrays: the copies into one then provably
  // do not write what the walk of the other reads, and its reads need not wait
  __shared__ V buf0[C::NV], buf1[C::NV];
  __shared__ int32_t soff[C::SX * C::SY][kStage2Rows + 1];
  if (gate && *gate == 0) return;
  // workgroup -> XCD region -> dual tile (padding workgroups return at once)
  const int ndx = (nxb + C::SX - 1) / C::SX, ndy = (nyb + C::SY - 1) / C::SY;
  const int nry = (ndy + C::RY - 1) / C::RY, nreg = ((ndx + C::RX - 1) / C::RX) * nry;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int reg = (slot / (C::RX * C::RY)) * 8 + xcd, loc = slot % (C::RX * C::RY);
  if (reg >= nreg) return;
  const int dx = (reg / nry) * C::RX + loc / C::RY, dy = (reg % nry) * C::RY + loc % C::RY;
  if (dx >= ndx || dy >= ndy) return;
  const int tid = threadIdx.x, sub = tid & 15, g = tid >> 4;
  // sub-tile st = (sx, sy): the positions where its 32 rows' outputs start
  for (int i = tid; i < C::SX * C::SY * (kStage2Rows + 1); i += C::NT) {
    const int st = i / (kStage2Rows + 1), j = i % (kStage2Rows + 1);
    const int xb = dx * C::SX + (st >> 1), yb = dy * C::SY + (st & 1);
    soff[st][j] = (xb < nxb && yb < nyb) ? (int32_t)tileoff[((int64_t)xb * nyb + yb) * (kStage2Rows + 1) + j] : 0;
  }
  const int64_t ct0 = (int64_t)(dx * C::SX) * nyb + dy * C::SY;
  const int64_t y0 = tiley[2 * ct0];
  const int64_t nyr = tiley[2 * ct0 + 1] + (dy * C::SY + 1 < nyb ? tiley[2 * ct0 + 3] : 0);
  __syncthreads();
  int cum[C::SX * C::SY + 1];
  cum[0] = 0;
#pragma unroll
  for (int st = 0; st < C::SX * C::SY; ++st) cum[st + 1] = cum[st] + (soff[st][kStage2Rows] - soff[st][0]);
  const int ntot = cum[C::SX * C::SY];
  const int64_t nch = (nkeys + C::KC - 1) / C::KC;
  const int wv = tid >> 6, ln = tid & 63;
  // copy chunk c into buffer bd: 256 rows of 256 bytes, four rows per wave
  // instruction (lane l: row 4 i + l / 16, bytes 16 (l % 16)); F1 rows past the
  // matrix read row 0 and S rows past the block its first row, and keys past
  // nkeys (whole 16-byte pieces, nkeys being a multiple of VEC) read the row's
  // first piece: their S partner is a zero of the row padding or they belong to
  // no output, so every staged value is finite and contributes nothing
  auto issue = [&](int64_t c, V *bd) {
    const int64_t kp = c * C::KC + (int64_t)(ln & 15) * C::VEC;
    for (int i = wv; i < (C::XT + C::YT) / 4; i += C::NT / 64) {
      const int r = 4 * i + (ln >> 4);
      const T *src;
      if (r < C::XT) {
        const int64_t x = (int64_t)dx * C::XT + r;
        src = F1 + (x < nx ? x : 0) * ld1 + (kp < nkeys ? kp : 0);
      } else {
        const int64_t yr = r - C::XT;
        src = S + (y0 + (yr < nyr ? yr : 0)) * ldS + kp;
      }
      lds_load_row16(src, bd + 4 * i * (C::CB / 16));
    }
  };
  for (int pass0 = 0; pass0 < ntot; pass0 += C::NG * C::OPG) {  // uniform
    const int cnt = min(C::OPG, max(0, (ntot - pass0 - g + C::NG - 1) / C::NG));
    // lane `sub` resolves output `sub` of its group: where its rows sit in a
    // chunk buffer (16-byte units) and its index
    int offa = 0, offb = 0;
    int64_t outi = 0;
    {
      const int idx = pass0 + g + C::NG * sub;
      if (sub < cnt) {
        int st = 0, cst = 0;  // the sub-tile holding output idx, and its first output
#pragma unroll
        for (int u = 1; u < C::SX * C::SY; ++u)
          if (idx >= cum[u]) {
            st = u;
            cst = cum[u];
          }
        const int q = soff[st][0] + (idx - cst);
        int lo = 0, hi = kStage2Rows;  // the row r with soff[st][r] <= q < soff[st][r + 1]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (soff[st][mid] <= q) lo = mid;
          else hi = mid;
        }
        offa = ((st >> 1) * kStage2Rows + lo) * (C::CB / 16);
        offb = (C::XT + (int)(yrows[q] - y0)) * (C::CB / 16);
        outi = perm[q];
      }
    }
    int oa[C::OPG], ob[C::OPG];
#pragma unroll
    for (int o = 0; o < C::OPG; ++o) {
      oa[o] = __shfl(offa, (tid & 48) + o, 64) + sub;
      ob[o] = __shfl(offb, (tid & 48) + o, 64) + sub;
    }
    T acc[C::OPG];
#pragma unroll
    for (int o = 0; o < C::OPG; ++o) acc[o] = T(0);
    __syncthreads();  // the previous pass's reads of the buffers are done
    issue(0, buf0);
    // chunk c walks buffer c mod 2 while chunk c + 1 is copied into the other;
    // the loop is unrolled by two so each half names its buffers at compile time
    auto walk = [&](int64_t c, const V *bc, V *bn) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk c have landed
      __syncthreads();                // everyone's have, and chunk c - 1 is walked
      if (c + 1 < nch) issue(c + 1, bn);
#pragma unroll
      for (int o = 0; o < C::OPG; ++o) {
        if (o < cnt) {
          const V a = bc[oa[o]];
          const V b = bc[ob[o]];
#pragma unroll
          for (int j = 0; j < C::VEC; ++j) acc[o] += a[j] * b[j];
        }
      }
    };
    for (int64_t c = 0; c < nch; c += 2) {
      walk(c, buf0, buf1);
      if (c + 1 < nch) walk(c + 1, buf1, buf0);
    }
    const int wn = wave_max_of_groups(cnt);
#pragma unroll
    for (int o = 0; o < C::OPG; ++o) {
      if (o < wn) acc[o] = row16_sum(acc[o]);
      if (sub == o && o < cnt) out[outi * ldi] = coef * acc[o];
    }
  }
}

// ---------------------------------------------------------------------------
// Stage 2 for blocks of R >= 4 right-hand sides, grouped by S row.  Each S
// element carries R values, so the roles swap: a 16-lane group owns one S row
// and holds that row's slice of the current key chunk (KPL keys x R values per
// lane) in registers, loaded once per chunk; the tile's F1 rows (at most
// kStage2MaxS of them) are staged in LDS, and every output of the row costs
// one 16-byte LDS read per KPL x R FMAs.  Tiles: 32 consecutive compact S rows
// x one block of F1 rows, outputs ordered by (tile, S row, F1 row).
template <class T, int R> struct S2yCfg {
  static_assert(R >= 4, "S-row grouped stage 2 is for blocks of 4 or more RHS");
  static constexpr int LPO = 16;                         // lanes per S row / output
  static constexpr int NG = kStage2Rows;                 // S rows per tile (32)
  static constexpr int NT = NG * LPO;                    // 512 threads
  static constexpr int KPL = 16 / (int)sizeof(T);        // keys per lane per chunk (one 16-byte F1 read)
  static constexpr int KC = LPO * KPL;                   // keys per chunk
  static constexpr int ACC = sizeof(T) == 4 ? 64 : 32;   // accumulators per lane
  static constexpr int OPG = ACC / R;                    // outputs per row per pass
  static constexpr int FROW = KC + 16 / (int)sizeof(T);  // LDS row: chunk + 16 B
  static_assert(KPL * sizeof(T) == 16, "one 16-byte LDS read per output and chunk");
};

template <class T, int R> struct S2ySmem {
  __attribute__((aligned(16))) T ftile[kStage2MaxS * S2yCfg<T, R>::FROW];
  unsigned char meta[S2yCfg<T, R>::NG][S2yCfg<T, R>::OPG];
};

template <class T, int R>
__device__ __forceinline__ void stage2y_tile(
    const T *__restrict__ F1, int64_t ld1, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tilex, const int32_t *__restrict__ tilemax,
    const uint8_t *__restrict__ grow, const int32_t *__restrict__ xrows,
    const int32_t *__restrict__ perm, int nxb, const T *__restrict__ S, int64_t ldS, int64_t nsr,
    int64_t nkeys, T coef, T *__restrict__ out, int64_t ldi, int64_t ldr, int t,
    S2ySmem<T, R> &sm) {
  typedef S2yCfg<T, R> C;
  typedef typename Vec16<T>::type V16;
  constexpr int VEC = 16 / sizeof(T);
  const int maxcnt = tilemax[t];
  if (maxcnt == 0) return;  // uniform: empty tile
  const int gb = t / nxb;
  const int64_t x0 = tilex[2 * t], nxr = tilex[2 * t + 1];
  const int sub = threadIdx.x % C::LPO, grp = threadIdx.x / C::LPO;
  const int gr = grow[(int64_t)t * C::NG + grp];  // rows by descending output count
  const int64_t yrow = (int64_t)gb * C::NG + gr;
  const int64_t qb = tileoff[(int64_t)t * (C::NG + 1) + gr];
  const int cnt = (int)(tileoff[(int64_t)t * (C::NG + 1) + gr + 1] - qb);
  const T *srow = S + (yrow < nsr ? yrow : 0) * ldS;
  const int64_t nch = (nkeys + C::KC - 1) / C::KC;
  // F1 rows start on 16-byte boundaries: whole pieces load as one vector
  const bool f1_vec = ld1 % VEC == 0 && reinterpret_cast<uintptr_t>(F1) % 16 == 0;
  for (int pass0 = 0; pass0 < maxcnt; pass0 += C::OPG) {
    const int npass = (cnt - pass0) < C::OPG ? (cnt - pass0) : C::OPG;  // may be <= 0
    __syncthreads();
    for (int o = sub; o < C::OPG; o += C::LPO)
      sm.meta[grp][o] = (o < npass) ? (unsigned char)(xrows[qb + pass0 + o] - x0) : 0;
    T acc[C::OPG][R];
#pragma unroll
    for (int o = 0; o < C::OPG; ++o)
#pragma unroll
      for (int r = 0; r < R; ++r) acc[o][r] = T(0);
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t k0 = c * C::KC;
      __syncthreads();
      // F1 rows of the tile, this chunk's keys (zero past the last key), in
      // 16-byte pieces
      {
        constexpr int PPR = C::KC / VEC;  // pieces per row
#pragma unroll 1
        for (int idx = threadIdx.x; idx < nxr * PPR; idx += C::NT) {
          const int row = idx / PPR, pc = idx - row * PPR;
          const int64_t k = k0 + pc * VEC;
          const T *src = F1 + (x0 + row) * ld1 + k;
          V16 v;
          if (f1_vec && k + VEC <= nkeys) {
            v = *reinterpret_cast<const V16 *>(src);
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = k + e < nkeys ? src[e] : T(0);
          }
          *reinterpret_cast<V16 *>(sm.ftile + row * C::FROW + pc * VEC) = v;
        }
      }
      // this lane's S slice: keys k0 + sub*KPL .. + KPL-1, R values each (KPL x R registers)
      T sv[C::KPL][R];
#pragma unroll
      for (int kk = 0; kk < C::KPL; ++kk) {
        const int64_t k = k0 + sub * C::KPL + kk;
        const bool ok = npass > 0 && k < nkeys;
#pragma unroll
        for (int r0 = 0; r0 < R; r0 += VEC) {
          V16 v;
          if (ok) {
            v = *reinterpret_cast<const V16 *>(srow + k * R + r0);
          } else {
#pragma unroll
            for (int u = 0; u < VEC; ++u) v[u] = T(0);
          }
#pragma unroll
          for (int u = 0; u < VEC; ++u) sv[kk][r0 + u] = v[u];
        }
      }
      __syncthreads();
#pragma unroll
      for (int o = 0; o < C::OPG; ++o) {
        if (o < npass) {
          const V16 f = *reinterpret_cast<const V16 *>(sm.ftile + (int)sm.meta[grp][o] * C::FROW +
                                                       sub * C::KPL);
#pragma unroll
          for (int kk = 0; kk < C::KPL; ++kk)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[o][r] += f[kk] * sv[kk][r];
        }
      }
    }
    // lane partial sums meet inside each 16-lane row; slots past every
    // group's count in this wave are skipped (wave-uniform bound)
    static_assert(C::LPO == 16, "one DPP row per output");
    const int wn = wave_max_of_groups(npass);
#pragma unroll
    for (int o = 0; o < C::OPG; ++o) {
      if (o < wn) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[o][r] = row16_sum(acc[o][r]);
      }
      if (sub == 0 && o < npass) {
        const int64_t i = perm[qb + pass0 + o];
#pragma unroll
        for (int r = 0; r < R; ++r) out[i * ldi + r * ldr] = coef * acc[o][r];
      }
    }
  }
}

// The same tile for blocks of 4 RHS with its key chunks pipelined: chunk c + 1
// is in flight while chunk c is walked.  The tile's F1 rows go from global
// memory straight into one of two LDS buffers (an F1 row's chunk is 16 pieces
// of 16 bytes, four rows per wave instruction) and each lane's S slice into one
// of two register sets.  Where F1 rows do not start on 16-byte boundaries, and
// for a piece that ends past the last key, the lanes stage their F1 pieces
// themselves through registers (zeros past the last key); S rows are whole
// zero-padded chunks.  With no staging registers in the walk a lane affords
// twice the accumulators (half the passes over the tile's chunks) at two waves
// per SIMD, and reads the F1 pieces of OB outputs together.  Every FMA is the
// one stage2y_tile makes, in the same order: the results are bitwise equal.
// (Measured, FP64 / FP32 4-RHS blocks on one MI355X, 200 000 outputs: 2000 x
// 500 grid 446 / 170 us -> 285 / 118 us, 1000 x 1000 grid 237 / 94 us -> 158 /
// 69 us.  The S chunks staged in LDS as well cost more LDS traffic than they
// saved: 329 / 194 us on the 2000 x 500 grid at four waves per SIMD.)
template <class T> struct S2ypCfg {
  typedef S2yCfg<T, 4> B;
  static constexpr int OPG = 2 * B::OPG;  // outputs per group per pass
  static constexpr int OB = 4;            // outputs per batch of F1 reads
  static constexpr int NP = kStage2MaxS * 16;  // F1 buffer: kStage2MaxS rows x 16 pieces
  static_assert(OPG % OB == 0 && OPG % 4 == 0, "whole batches, whole 32-bit words of meta");
};

__host__ __device__ inline bool stage2y_rows16(const void *F1, int64_t ld1, size_t es) {
  return reinterpret_cast<uintptr_t>(F1) % 16 == 0 && (ld1 * (int64_t)es) % 16 == 0;
}

template <class T>
__device__ __forceinline__ void stage2y_tile_pipelined(
    const T *__restrict__ F1, int64_t ld1, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tilex, const int32_t *__restrict__ tilemax,
    const uint8_t *__restrict__ grow, const int32_t *__restrict__ xrows,
    const int32_t *__restrict__ perm, int nxb, const T *__restrict__ S, int64_t ldS, int64_t nsr,
    int64_t nkeys, T coef, T *__restrict__ out, int64_t ldi, int64_t ldr, int t,
    typename Vec16<T>::type *fb0, typename Vec16<T>::type *fb1, unsigned char (*meta)[S2ypCfg<T>::OPG]) {
  constexpr int R = 4;
  typedef S2yCfg<T, R> C;
  typedef S2ypCfg<T> P;
  typedef typename Vec16<T>::type V16;
  constexpr int VEC = 16 / sizeof(T);
  static_assert(C::KC * sizeof(T) == 256, "an F1 row's chunk is 16 pieces of 16 bytes");
  static_assert(C::KPL * R == 4 * VEC, "a lane's S slice is four pieces");
  const int maxcnt = tilemax[t];
  if (maxcnt == 0) return;  // uniform: empty tile
  const int gb = t / nxb;
  const int64_t x0 = tilex[2 * t], nxr = tilex[2 * t + 1];
  const int sub = threadIdx.x % C::LPO, grp = threadIdx.x / C::LPO;
  const int gr = grow[(int64_t)t * C::NG + grp];  // rows by descending output count
  const int64_t qb = tileoff[(int64_t)t * (C::NG + 1) + gr];
  const int cnt = (int)(tileoff[(int64_t)t * (C::NG + 1) + gr + 1] - qb);
  const int nch = (int)((nkeys + C::KC - 1) / C::KC);
  const int nk = (int)nkeys;
  const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
  const int nri = (int)((nxr + 3) / 4);  // wave instructions per F1 chunk, four rows each
  const bool rows16 = stage2y_rows16(F1, ld1, sizeof(T));
  // chunk c of the tile's F1 rows into bd (row r at pieces 16 r .. 16 r + 15)
  auto issue = [&](int c, V16 *bd) {
    const int kp = c * C::KC + (ln & 15) * VEC;
    for (int i = wv; i < nri; i += C::NT / 64) {
      const int r = 4 * i + (ln >> 4);
      const T *src = F1 + (x0 + (r < nxr ? r : 0)) * ld1;
      V16 *dst = bd + 4 * i * 16;  // the wave's base: lane ln lands at dst[ln]
      if (rows16 && kp + VEC <= nk) {
        lds_load_row16(src + kp, dst);
      } else {
        V16 v;
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = kp + e < nk ? src[kp + e] : T(0);
        dst[ln] = v;
      }
    }
  };
  // this lane's S slice of chunk c: keys c KC + sub KPL .. + KPL - 1, R values
  // each (rows past the buffer read row 0: they have no outputs)
  const int64_t yrow = (int64_t)gb * C::NG + gr;
  const T *sl = S + (yrow < nsr ? yrow : 0) * ldS + sub * (C::KPL * R);
  auto sload = [&](int c, T (&v)[C::KPL][R]) {
#pragma unroll
    for (int u0 = 0; u0 < 4; ++u0) {
      const V16 w = *reinterpret_cast<const V16 *>(sl + (int64_t)c * (C::KC * R) + u0 * VEC);
#pragma unroll
      for (int u = 0; u < VEC; ++u) v[(u0 * VEC + u) / R][(u0 * VEC + u) % R] = w[u];
    }
  };
  for (int pass0 = 0; pass0 < maxcnt; pass0 += P::OPG) {
    const int npass = (cnt - pass0) < P::OPG ? (cnt - pass0) : P::OPG;  // may be <= 0
    __syncthreads();  // the previous pass's reads of the buffers and meta are done
    for (int o = sub; o < P::OPG; o += C::LPO)
      meta[grp][o] = (o < npass) ? (unsigned char)(xrows[qb + pass0 + o] - x0) : 0;
    // this group's F1 rows for the pass, packed four to a register
    __syncthreads();
    unsigned mp[P::OPG / 4];
#pragma unroll
    for (int q = 0; q < P::OPG / 4; ++q) mp[q] = *reinterpret_cast<const unsigned *>(&meta[grp][4 * q]);
    T acc[P::OPG][R];
#pragma unroll
    for (int o = 0; o < P::OPG; ++o)
#pragma unroll
      for (int r = 0; r < R; ++r) acc[o][r] = T(0);
    T sa[C::KPL][R], sb[C::KPL][R];
    issue(0, fb0);
    sload(0, sa);
    // chunk c walks F1 buffer and S set c mod 2 while chunk c + 1 comes into
    // the others; the loop is unrolled by two so each half names its buffers
    // at compile time
    auto walk = [&](int c, const V16 *bc, V16 *bn, T (&sv)[C::KPL][R], T (&svn)[C::KPL][R]) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies and loads of chunk c have landed
      __syncthreads();                // everyone's have, and chunk c - 1 is walked
      if (c + 1 < nch) {
        issue(c + 1, bn);
        sload(c + 1, svn);
      }
      // outputs in batches of OB behind one branch, their F1 reads in flight
      // together; slots past npass read F1 row 0 (meta is 0 there) into
      // accumulators that are never stored
#pragma unroll
      for (int o0 = 0; o0 < P::OPG; o0 += P::OB) {
        if (o0 < npass) {
          V16 f[P::OB];
#pragma unroll
          for (int q = 0; q < P::OB; ++q) {
            const int o = o0 + q;
            f[q] = bc[(int)((mp[o >> 2] >> (8 * (o & 3))) & 0xffu) * 16 + sub];
          }
#pragma unroll
          for (int q = 0; q < P::OB; ++q)
#pragma unroll
            for (int kk = 0; kk < C::KPL; ++kk)
#pragma unroll
              for (int r = 0; r < R; ++r) acc[o0 + q][r] += f[q][kk] * sv[kk][r];
        }
      }
    };
    for (int c = 0; c < nch; c += 2) {
      walk(c, fb0, fb1, sa, sb);
      if (c + 1 < nch) walk(c + 1, fb1, fb0, sb, sa);
    }
    // lane partial sums meet inside each 16-lane row; slots past every
    // group's count in this wave are skipped (wave-uniform bound)
    const int wn = wave_max_of_groups(npass);
#pragma unroll
    for (int o = 0; o < P::OPG; ++o) {
      if (o < wn) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[o][r] = row16_sum(acc[o][r]);
      }
      if (sub == 0 && o < npass) {
        const int64_t i = perm[qb + pass0 + o];
#pragma unroll
        for (int r = 0; r < R; ++r) out[i * ldi + r * ldr] = coef * acc[o][r];
      }
    }
  }
}

template <class T, int R>
__global__ __launch_bounds__(kStage2Rows * 16) __attribute__((amdgpu_waves_per_eu(4))) void stage2y_kernel(
    const T *__restrict__ F1, int64_t ld1, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tilex, const int32_t *__restrict__ tilemax,
    const uint8_t *__restrict__ grow, const int32_t *__restrict__ xrows,
    const int32_t *__restrict__ perm, int nxb, const T *__restrict__ S, int64_t ldS, int64_t nsr,
    int64_t nkeys, T coef, T *__restrict__ out, int64_t ldi, int64_t ldr,
    const int *__restrict__ gate) {
  __shared__ S2ySmem<T, R> sm;
  if (gate && *gate == 0) return;
  stage2y_tile<T, R>(F1, ld1, tileoff, tilex, tilemax, grow, xrows, perm, nxb, S, ldS, nsr, nkeys, coef,
                     out, ldi, ldr, blockIdx.x, sm);
}

template <class T>
__global__ __launch_bounds__(kStage2Rows * 16) __attribute__((amdgpu_waves_per_eu(2))) void stage2y_pipelined_kernel(
    const T *__restrict__ F1, int64_t ld1, const int64_t *__restrict__ tileoff,
    const int32_t *__restrict__ tilex, const int32_t *__restrict__ tilemax,
    const uint8_t *__restrict__ grow, const int32_t *__restrict__ xrows,
    const int32_t *__restrict__ perm, int nxb, const T *__restrict__ S, int64_t ldS, int64_t nsr,
    int64_t nkeys, T coef, T *__restrict__ out, int64_t ldi, int64_t ldr,
    const int *__restrict__ gate) {
  __shared__ typename Vec16<T>::type fb0[S2ypCfg<T>::NP], fb1[S2ypCfg<T>::NP];
  __shared__ __attribute__((aligned(4))) unsigned char meta[S2yCfg<T, 4>::NG][S2ypCfg<T>::OPG];
  if (gate && *gate == 0) return;
  stage2y_tile_pipelined<T>(F1, ld1, tileoff, tilex, tilemax, grow, xrows, perm, nxb, S, ldS, nsr, nkeys,
                            coef, out, ldi, ldr, blockIdx.x, fb0, fb1, meta);
}

// ---------------------------------------------------------------------------
// One-factor terms: g[x*R + r] = sum_k F(x,k)^{1|2} s[k*R + r]; one wave per row.
template <class T, bool SQ>
__global__ __launch_bounds__(256) void gemv_kernel(const T *__restrict__ F, int64_t ldf,
                                                   int64_t nrows, int64_t ncols,
                                                   const T *__restrict__ s, int R,
                                                   T *__restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int64_t x = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= nrows) return;
  const T *frow = F + x * ldf;
  for (int r = 0; r < R; ++r) {
    T acc = T(0);
    for (int64_t k = lane; k < ncols; k += WAVE) {
      T f = frow[k];
      if (SQ) f = f * f;
      acc += f * s[k * R + r];
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) g[x * R + r] = acc;
  }
}

// t[i*R + r] = g[sel[i]*R + r]
template <class T>
__global__ void gather_rows_kernel(const T *__restrict__ g, const int32_t *__restrict__ sel,
                                   int64_t n, int R, T *__restrict__ t) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t x = sel[i];
  for (int r = 0; r < R; ++r) t[i * R + r] = g[x * R + r];
}

// Cartesian sparse-match term: t[i] = sum_{p in seg(kv_i)} F[x_i, other_p] vs[p]
// (kv_i >= nkeys: the object never occurs on the input side -> 0).  A
// 16-lane group per output strides the key segment; the lanes' partial sums
// meet in a fixed butterfly.
template <class T>
__global__ __launch_bounds__(256) void match_kernel(const T *__restrict__ F, int64_t ldf,
                                                    const int32_t *__restrict__ xsel,
                                                    const int32_t *__restrict__ ksel, int64_t n,
                                                    const int64_t *__restrict__ seg,
                                                    const int32_t *__restrict__ other,
                                                    const T *__restrict__ vs, int64_t nkeys, int R,
                                                    T *__restrict__ t) {
  constexpr int G = 16;
  const int sub = threadIdx.x % G;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const bool live = i < n;
  int64_t p0 = 0, p1 = 0;
  const T *frow = F;
  if (live) {
    const int64_t kv = ksel[i];
    frow = F + (int64_t)xsel[i] * ldf;
    if (kv < nkeys) { p0 = seg[kv]; p1 = seg[kv + 1]; }
  }
  for (int r = 0; r < R; ++r) {
    T acc = T(0);
    for (int64_t p = p0 + sub; p < p1; p += G) acc += frow[other[p]] * vs[p * R + r];
#pragma unroll
    for (int off = 1; off < G; off <<= 1) acc += __shfl_xor(acc, off);
    if (live && sub == 0) t[i * R + r] = acc;
  }
}

// Cartesian match terms with the F row staged in LDS: one block per F row x
// stages F[x, :] and its 16-lane groups walk the outputs of that row, each
// summing its key segment; the gathers F[x, other_p] then hit LDS instead of
// scattered cache lines.  All R right-hand sides share one walk.
template <class T, int R>
__global__ __launch_bounds__(256) void match_row_kernel(const T *__restrict__ F, int64_t ldf,
                                                        int64_t ncols,
                                                        const int32_t *__restrict__ operm,
                                                        const int64_t *__restrict__ xoff,
                                                        const int32_t *__restrict__ ksel,
                                                        const int64_t *__restrict__ seg,
                                                        const int32_t *__restrict__ other,
                                                        const T *__restrict__ vs, int64_t nkeys,
                                                        T *__restrict__ t) {
  extern __shared__ __attribute__((aligned(16))) unsigned char match_smem[];
  T *row = reinterpret_cast<T *>(match_smem);
  constexpr int G = 16;
  const int64_t x = blockIdx.x;
  const int64_t q0 = xoff[x], q1 = xoff[x + 1];
  if (q0 == q1) return;  // uniform: no outputs on this row
  const T *frow = F + x * ldf;
  for (int64_t c = threadIdx.x; c < ncols; c += 256) row[c] = frow[c];
  __syncthreads();
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  for (int64_t q = q0 + grp; q < q1; q += 256 / G) {
    const int64_t i = operm[q];
    const int64_t kv = ksel[i];
    int64_t p0 = 0, p1 = 0;
    if (kv < nkeys) { p0 = seg[kv]; p1 = seg[kv + 1]; }
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
    for (int64_t p = p0 + sub; p < p1; p += G) {
      const T f = row[other[p]];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += f * vs[p * R + r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T v = acc[r];
#pragma unroll
      for (int off = 1; off < G; off <<= 1) v += __shfl_xor(v, off);
      if (sub == 0) t[i * R + r] = v;
    }
  }
}

// Ft[o*ldt + y] = F[y*ldf + o]  (32x32 LDS tiles)
template <class T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ F, int64_t ldf,
                                                        int64_t rows, int64_t cols,
                                                        T *__restrict__ Ft, int64_t ldt) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int j = ty; j < 32; j += 8) {
    int64_t r = r0 + j, c = c0 + tx;
    if (r < rows && c < cols) tile[j][tx] = F[r * ldf + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    int64_t c = c0 + j, r = r0 + tx;
    if (r < rows && c < cols) Ft[c * ldt + r] = tile[tx][j];
  }
}

// U_o[i + r*ldu] = sum_k coef[o][k] * t_k[i*R + r]
template <class T>
__global__ void combine_kernel(CombineArgs<T> a, int64_t n, int R, T *__restrict__ U, int64_t ldu,
                               int64_t block_stride) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int o = 0; o < a.nout; ++o) {
    T *Uo = U + o * block_stride;
    for (int r = 0; r < R; ++r) {
      T acc = T(0);
      for (int k = 0; k < a.nterms; ++k) {
        const T c = a.coef[o][k];
        if (c != T(0)) acc += c * a.t[k][i * R + r];
      }
      Uo[i + r * ldu] = acc;
    }
  }
}

template <class T>
__global__ void fill_kernel(T *__restrict__ U, int64_t rows, int64_t cols, int64_t ld, T val) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  int64_t c = idx / rows, r = idx - c * rows;
  U[r + c * ld] = val;
}

// ---------------------------------------------------------------------------
// Grouped kernels: one launch over the blocks of many independent problems.
// Each workgroup reads its (problem, local block) item and the problem's
// descriptor, then runs the same block body as the single-product kernels.
// Problems whose active flag is 0 are skipped as a whole.
static constexpr int kGroupPackBlock = 256;

template <class T>
__global__ __launch_bounds__(256) void group_pack_kernel(const GroupDesc<T> *__restrict__ desc,
                                                         const GroupItem *__restrict__ items, int R,
                                                         int64_t r0,
                                                         const uint8_t *__restrict__ active) {
  const GroupItem it = items[blockIdx.x];
  if (active && !active[it.p]) return;
  const GroupDesc<T> &d = desc[it.p];
  const int64_t pos = (int64_t)it.li * kGroupPackBlock + threadIdx.x;
  if (pos >= d.n_in) return;
  const int64_t j = d.perm_in[pos];
  const T *V = d.V + r0 * d.ldv;
  for (int r = 0; r < R; ++r) d.vs[pos * R + r] = V[j + r * d.ldv];
}

template <class T, int R>
__global__ __launch_bounds__(256) void group_stage1_kernel(const GroupDesc<T> *__restrict__ desc,
                                                           const GroupItem *__restrict__ items,
                                                           const uint8_t *__restrict__ active) {
  constexpr int NARROW = 64 * (S1Cfg<T, R>::KB * R + 1), WIDE = S1WideCfg<T, R, 1>::STG;
  __shared__ T stg[NARROW > WIDE ? NARROW : WIDE];
  const GroupItem it = items[blockIdx.x];
  if (active && !active[it.p]) return;
  const GroupDesc<T> &d = desc[it.p];
  const int nkb = (int)d.nkb;
  const int kb = it.li % nkb, rb = it.li / nkb;
  if (d.row0 >= 0)  // uniform: the problem's walk
    stage1_wide_block<T, R, 1>(d.Fc, d.ldc, d.row0, d.nrows, d.seg, d.other, d.vs, d.nkeys, d.S,
                               sbuf_row_ld<T>(d.nkeys, R), kb, rb, stg);
  else
    stage1_block<T, R>(d.Fc, d.ldc, d.rows, d.nrows, d.seg, d.other, d.vs, d.nkeys, d.S,
                       sbuf_row_ld<T>(d.nkeys, R), kb, rb, stg);
}

template <class T, int R>
__global__ __launch_bounds__(S1SliceCfg<T>::NT) void group_stage1_slice_kernel(
    const GroupDesc<T> *__restrict__ desc, const GroupItem *__restrict__ items,
    const uint8_t *__restrict__ active) {
  extern __shared__ __attribute__((aligned(16))) unsigned char s1s_lds[];
  const GroupItem it = items[blockIdx.x];
  if (active && !active[it.p]) return;
  const GroupDesc<T> &d = desc[it.p];
  const int64_t kr = it.li % d.nkr, rb = it.li / d.nkr;
  stage1_slice_block<T, R>(d.Fc, d.ldc, d.row0, d.nrows, d.seg, d.other, d.vs, d.nkeys, d.nother, d.S,
                           sbuf_row_ld<T>(d.nkeys, R), d.kpr, kr, rb, s1s_lds);
}

template <class T, int R>
__global__ __launch_bounds__(kStage2Rows * 16) void group_stage2_kernel(const GroupDesc<T> *__restrict__ desc,
                                                           const GroupItem *__restrict__ items,
                                                           int64_t r0,
                                                           const uint8_t *__restrict__ active) {
  __shared__ S2Smem<T, R> sm;
  const GroupItem it = items[blockIdx.x];
  if (active && !active[it.p]) return;
  const GroupDesc<T> &d = desc[it.p];
  stage2_tile<T, R>(d.F1, d.ld1, d.nx, d.tileoff[0], d.tiley[0], d.tilemax[0], d.grow[0], d.yrows[0],
                    d.perm_out[0], (int)d.nyb[0], d.S, sbuf_row_ld<T>(d.nkeys, R), d.nkeys, T(1),
                    d.U + r0 * d.ldu, 1, d.ldu, it.li, sm);
}

template <class T, int R>
__global__ __launch_bounds__(kStage2Rows * 16) __attribute__((amdgpu_waves_per_eu(4))) void group_stage2y_kernel(const GroupDesc<T> *__restrict__ desc,
                                                            const GroupItem *__restrict__ items,
                                                            int64_t r0,
                                                            const uint8_t *__restrict__ active) {
  __shared__ S2ySmem<T, R> sm;
  const GroupItem it = items[blockIdx.x];
  if (active && !active[it.p]) return;
  const GroupDesc<T> &d = desc[it.p];
  stage2y_tile<T, R>(d.F1, d.ld1, d.tileoff[1], d.tiley[1], d.tilemax[1], d.grow[1], d.yrows[1],
                     d.perm_out[1],
                     (int)d.nyb[1], d.S, sbuf_row_ld<T>(d.nkeys, R), d.nrows, d.nkeys, T(1),
                     d.U + r0 * d.ldu, 1, d.ldu, it.li, sm);
}

template <class T>
__global__ __launch_bounds__(kStage2Rows * 16) __attribute__((amdgpu_waves_per_eu(2))) void group_stage2y_pipelined_kernel(
    const GroupDesc<T> *__restrict__ desc, const GroupItem *__restrict__ items, int64_t r0,
    const uint8_t *__restrict__ active) {
  __shared__ typename Vec16<T>::type fb0[S2ypCfg<T>::NP], fb1[S2ypCfg<T>::NP];
  __shared__ __attribute__((aligned(4))) unsigned char meta[S2yCfg<T, 4>::NG][S2ypCfg<T>::OPG];
  const GroupItem it = items[blockIdx.x];
  if (active && !active[it.p]) return;
  const GroupDesc<T> &d = desc[it.p];
  stage2y_tile_pipelined<T>(d.F1, d.ld1, d.tileoff[1], d.tiley[1], d.tilemax[1], d.grow[1], d.yrows[1],
                            d.perm_out[1], (int)d.nyb[1], d.S, sbuf_row_ld<T>(d.nkeys, 4), d.nrows, d.nkeys, T(1),
                            d.U + r0 * d.ldu, 1, d.ldu, it.li, fb0, fb1, meta);
}

// ===========================================================================
// Launchers
// ===========================================================================
static inline dim3 grid1(int64_t n, int bs) { return dim3((unsigned)ceil_div(n, bs)); }

template <class T>
void launch_pack_v(const T *V, int64_t ldv, const int32_t *perm, int64_t n, int R, T *vs,
                   hipStream_t s, const int *gate) {
  if (n <= 0) return;
  pack_v_kernel<T><<<grid1(n, 256), 256, 0, s>>>(V, ldv, perm, n, R, vs, gate);
}

template <class T>
void launch_segsum(const int64_t *seg, const T *vs, int64_t nkeys, int R, T *out, hipStream_t s) {
  if (nkeys <= 0) return;
  segsum_kernel<T><<<grid1(nkeys, 256), 256, 0, s>>>(seg, vs, nkeys, R, out);
}

template <class T, int R, int KPW>
static void stage1_rk(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, const int64_t *seg,
                      const int32_t *other, const T *vs, int64_t nkeys, T *S, int64_t ldS,
                      hipStream_t s, const int *gate) {
  typedef S1Cfg<T, R, KPW> C;
  dim3 grid((unsigned)ceil_div(nkeys, C::KB), (unsigned)ceil_div(nrows, 64));
  stage1_kernel<T, R, KPW><<<grid, 256, 0, s>>>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, gate);
}

// Launch knobs of stage 1: the tuned constants (tuning.h), overridable through
// GVT_STAGE1_KPW (1, 2 or 4 keys per wave) and GVT_STAGE1_WIDE (0 / 1: several
// rows per lane over contiguous rows) for tuning sweeps.  The environment is
// read when a plan is built, not per launch.
static std::atomic<int> g_s1_kpw{kStage1KeysPerWave}, g_s1_wide{kStage1Wide};

// Stage-2 XCD order: -1 chosen per launch, 0 by S block, 1 by F1 block (GVT_STAGE2_XCD).
static std::atomic<int> g_s2_xcd{-1};
// Stage 2 over dual tiles at low output density: -1 chosen per launch, 0 off,
// 1 wherever it applies (GVT_STAGE2_DUAL).
static std::atomic<int> g_s2_dual{-1};
// Stage 1 over an F2 slice resident in LDS where it fits (tuned kStage1Slice;
// GVT_STAGE1_SLICE overrides), with about this many workgroups per launch
// (kStage1SliceWgs; GVT_STAGE1_SLICE_WGS).
static std::atomic<int> g_s1_slice{kStage1Slice}, g_s1_slice_wgs{kStage1SliceWgs};
// Stage 2 of 4-RHS blocks with its key chunks pipelined (GVT_STAGE2Y_PIPELINED=0
// switches it off).
static std::atomic<int> g_s2y_pipe{1};
static int stage2y_use_pipelined() { return g_s2y_pipe.load(std::memory_order_relaxed); }

void refresh_launch_knobs() {
  const char *e9 = std::getenv("GVT_STAGE2Y_PIPELINED");
  g_s2y_pipe.store(e9 ? (std::atoi(e9) != 0) : 1, std::memory_order_relaxed);
  const char *e8 = std::getenv("GVT_STAGE2_DUAL");
  g_s2_dual.store(e8 ? (std::atoi(e8) != 0) : -1, std::memory_order_relaxed);
  const char *e6 = std::getenv("GVT_STAGE1_SLICE");
  g_s1_slice.store(e6 ? (std::atoi(e6) != 0) : kStage1Slice, std::memory_order_relaxed);
  const char *e7 = std::getenv("GVT_STAGE1_SLICE_WGS");
  g_s1_slice_wgs.store(e7 ? std::max(1, std::atoi(e7)) : kStage1SliceWgs, std::memory_order_relaxed);
  const char *e5 = std::getenv("GVT_STAGE2_XCD");
  g_s2_xcd.store(e5 ? (std::atoi(e5) != 0) : -1, std::memory_order_relaxed);
  const char *e1 = std::getenv("GVT_STAGE1_KPW");
  const int k = e1 ? std::atoi(e1) : kStage1KeysPerWave;
  g_s1_kpw.store((k == 1 || k == 2 || k == 4) ? k : 4, std::memory_order_relaxed);
  const char *e4 = std::getenv("GVT_STAGE1_WIDE");
  g_s1_wide.store(e4 ? (std::atoi(e4) != 0) : kStage1Wide, std::memory_order_relaxed);
}

static int stage1_kpw() { return g_s1_kpw.load(std::memory_order_relaxed); }
static bool stage1_use_slice() { return g_s1_slice.load(std::memory_order_relaxed) != 0; }
static bool stage1_use_wide() { return g_s1_wide.load(std::memory_order_relaxed) != 0; }
bool stage1_wide_enabled() { return stage1_use_wide(); }

template <class T, int R>
static void stage1_r(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, const int64_t *seg,
                     const int32_t *other, const T *vs, int64_t nkeys, T *S, int64_t ldS,
                     hipStream_t s, const int *gate) {
  switch (stage1_kpw()) {
    case 1: stage1_rk<T, R, 1>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
    case 2: stage1_rk<T, R, 2>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
    default: stage1_rk<T, R, 4>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
  }
}

template <class T, int R, int KPW>
static void stage1_wide_rk(const T *Fc, int64_t ldc, int64_t row0, int64_t nrows, const int64_t *seg,
                           const int32_t *other, const T *vs, int64_t nkeys, int64_t nother, T *S,
                           int64_t ldS, hipStream_t s, const int *gate) {
  typedef S1WideCfg<T, R, KPW> C;
  const int64_t nkb = ceil_div(nkeys, C::KB), nrb = ceil_div(nrows, C::ROWS);
  // XCD-grouped order when the F2 rows the walk reads exceed one XCD's L2
  // (measured: fused four-kind workload, 5 000 x 5 000 F2, stage 1 -21% FP32,
  // -24% FP64; ridge workload, 2 MB F2, +9% FP64: there every L2 holds all of F2)
  if ((double)nrows * (double)nother * sizeof(T) > kL2BytesPerXcd) {
    const int64_t per = ceil_div(nkb * nrb, 8);
    GVT_REQUIRE(8 * per < ((int64_t)1 << 31), GVT_ERR_ARG, "stage 1: too many blocks");
    stage1_wide_kernel<T, R, KPW><<<(unsigned)(8 * per), 256, 0, s>>>(
        Fc, ldc, row0, nrows, seg, other, vs, nkeys, S, ldS, nkb, per, gate);
  } else {
    stage1_wide_kernel<T, R, KPW><<<dim3((unsigned)nkb, (unsigned)nrb), 256, 0, s>>>(
        Fc, ldc, row0, nrows, seg, other, vs, nkeys, S, ldS, nkb, 0, gate);
  }
}

template <class T>
static void stage1_wide(const T *Fc, int64_t ldc, int64_t row0, int64_t nrows, const int64_t *seg,
                        const int32_t *other, const T *vs, int64_t nkeys, int64_t nother, int R, T *S,
                        int64_t ldS, hipStream_t s, const int *gate) {
#define GVT_S1W(RR, KK) stage1_wide_rk<T, RR, KK>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, s, gate)
  switch (R * 16 + stage1_kpw()) {
    case 16 + 1: GVT_S1W(1, 1); return;
    case 16 + 2: GVT_S1W(1, 2); return;
    case 16 + 4: GVT_S1W(1, 4); return;
    case 32 + 1: GVT_S1W(2, 1); return;
    case 32 + 2: GVT_S1W(2, 2); return;
    case 32 + 4: GVT_S1W(2, 4); return;
    case 64 + 1: GVT_S1W(4, 1); return;
    case 64 + 2: GVT_S1W(4, 2); return;
    case 64 + 4: GVT_S1W(4, 4); return;
    case 128 + 1: GVT_S1W(8, 1); return;
    case 128 + 2: GVT_S1W(8, 2); return;
    case 128 + 4: GVT_S1W(8, 4); return;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in stage 1"};
  }
#undef GVT_S1W
}

// The slice walk: a grid of (key ranges, row blocks), about one workgroup per
// CU (one fits at a time: the slices take up to 150 KB of LDS, and each
// workgroup copies its slice once; ridge workload, FP64: 23 us with 256
// workgroups, 26 with 512 or 1024), key ranges in whole rounds of the
// workgroup's 64 groups where the keys allow.
template <class T, int R>
static void stage1_slice_r(const T *Fc, int64_t ldc, int64_t row0, int64_t nrows, const int64_t *seg,
                           const int32_t *other, const T *vs, int64_t nkeys, int64_t nother, T *S,
                           int64_t ldS, hipStream_t s, const int *gate) {
  typedef S1SliceCfg<T> C;
  const int64_t nrb = ceil_div(nrows, (int64_t)C::RB);
  const int64_t want = std::max<int64_t>(1, ceil_div((int64_t)g_s1_slice_wgs.load(std::memory_order_relaxed), nrb));
  const int64_t nkr = std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(nkeys, (int64_t)64)));
  const int64_t kpr = ceil_div(nkeys, nkr);
  const size_t lds = (size_t)nother * 256;
  static std::once_flag once;
  std::call_once(once, [] {
    // allow the slices' dynamic LDS (the launch reports an error if the device has less)
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&stage1_slice_kernel<T, R>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kS1SliceMaxCols * 256)) != hipSuccess)
      (void)hipGetLastError();
  });
  GVT_REQUIRE(nrb < 65536, GVT_ERR_ARG, "internal: too many stage-1 row blocks");
  stage1_slice_kernel<T, R><<<dim3((unsigned)ceil_div(nkeys, kpr), (unsigned)nrb), C::NT, lds, s>>>(
      Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, kpr, gate);
}

template <class T>
static bool stage1_slice(const T *Fc, int64_t ldc, int64_t row0, int64_t nrows, const int64_t *seg,
                         const int32_t *other, const T *vs, int64_t nkeys, int64_t nother, int R, T *S,
                         int64_t ldS, hipStream_t s, const int *gate) {
  switch (R) {
    case 1: stage1_slice_r<T, 1>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, s, gate); return true;
    case 2: stage1_slice_r<T, 2>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, s, gate); return true;
    case 4: stage1_slice_r<T, 4>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, s, gate); return true;
    case 8: stage1_slice_r<T, 8>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, S, ldS, s, gate); return true;
    default: return false;
  }
}

template <class T>
static void stage1_direct(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows,
                          const int64_t *seg, const int32_t *other, const T *vs, int64_t nkeys, int R,
                          T *S, int64_t ldS, hipStream_t s, const int *gate) {
  if (nrows <= 0) return;
  switch (R) {
    case 1: stage1_r<T, 1>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
    case 2: stage1_r<T, 2>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
    case 4: stage1_r<T, 4>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
    case 8: stage1_r<T, 8>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, ldS, s, gate); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in stage 1"};
  }
}

template <class T>
void launch_stage1(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, int64_t row0,
                   const int64_t *seg, const int32_t *other, int64_t nother, const T *vs,
                   int64_t nkeys, int R, T *S, int64_t ldS, hipStream_t s, const int *gate) {
  if (nrows <= 0 || nkeys <= 0) return;
  // a contiguous range of at least one row block whose F2 columns' slices fit
  // in LDS: the slice walk
  if (row0 >= 0 && stage1_use_slice() && nrows >= S1SliceCfg<T>::RB && nother >= 1 &&
      nother <= kS1SliceMaxCols &&
      stage1_slice<T>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, R, S, ldS, s, gate))
    return;
  // a contiguous range of at least 16 bytes of rows: several rows per lane
  if (row0 >= 0 && stage1_use_wide() && nrows >= 16 / (int64_t)sizeof(T)) {
    stage1_wide<T>(Fc, ldc, row0, nrows, seg, other, vs, nkeys, nother, R, S, ldS, s, gate);
    return;
  }
  stage1_direct<T>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, R, S, ldS, s, gate);
}

template <class T>
void launch_colscale(const T *F, int64_t ldf, const int32_t *rows, int64_t nrows, const T *sv,
                     int64_t nkeys, int R, T *S, int64_t ldS, hipStream_t s) {
  if (nrows * nkeys <= 0) return;
  colscale_kernel<T><<<grid1(nrows * (ldS / R), 256), 256, 0, s>>>(F, ldf, rows, nrows, sv, nkeys, R, S,
                                                                   ldS);
}

template <class T>
void launch_stage2(const T *F1, int64_t ld1, int64_t nx, const int64_t *tileoff, const int32_t *tiley,
                   const int32_t *tilemax, const uint8_t *grow, int64_t ntiles, int nyb,
                   const int32_t *yrows, const int32_t *perm, const T *S, int64_t ldS, int64_t nsrows,
                   int64_t nkeys, int R, T coef, T *out, int64_t ldi, int64_t ldr, hipStream_t s,
                   const int *gate) {
  if (ntiles <= 0) return;
  // XCDs by F1 block re-read S once per F1 block: from the memory-side cache
  // while F1 and S fit in it together, from HBM otherwise, where XCDs by S
  // block (each keeping its slice of S) cost less
  const int xo = g_s2_xcd.load(std::memory_order_relaxed);
  const double bytes = (double)sizeof(T) * ((double)nx * (double)nkeys + (double)nsrows * (double)ldS);
  const int by_f1 = xo >= 0 ? xo : bytes <= kMallBytes;
  const int nxb = (int)(ntiles / nyb);
  dim3 grid((unsigned)(by_f1 ? (int64_t)ceil_div(nxb, 8) * 8 * nyb : ntiles));
  const int nt = S2Cfg<T, 1>::NT;
  switch (R) {
    case 1: stage2_kernel<T, 1><<<grid, nt, 0, s>>>(F1, ld1, nx, tileoff, tiley, tilemax, grow, yrows, perm, nyb, S, ldS, nkeys, coef, out, ldi, ldr, gate, nxb, by_f1); break;
    case 2: stage2_kernel<T, 2><<<grid, nt, 0, s>>>(F1, ld1, nx, tileoff, tiley, tilemax, grow, yrows, perm, nyb, S, ldS, nkeys, coef, out, ldi, ldr, gate, nxb, by_f1); break;
    case 4: stage2_kernel<T, 4><<<grid, nt, 0, s>>>(F1, ld1, nx, tileoff, tiley, tilemax, grow, yrows, perm, nyb, S, ldS, nkeys, coef, out, ldi, ldr, gate, nxb, by_f1); break;
    case 8: stage2_kernel<T, 8><<<grid, nt, 0, s>>>(F1, ld1, nx, tileoff, tiley, tilemax, grow, yrows, perm, nyb, S, ldS, nkeys, coef, out, ldi, ldr, gate, nxb, by_f1); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in stage 2"};
  }
}

// Stage 2 over dual tiles where it applies: one RHS, F1 rows 16-byte aligned
// (global-to-LDS copies), nkeys a multiple of the vector length, and a low
// output density (auto: at most 700 outputs per dual tile on average, so one
// pass of 1 024 output slots serves a tile).  Returns false where it does not.
template <class T>
bool launch_stage2_dual(const T *F1, int64_t ld1, int64_t nx, const int64_t *tileoff, const int32_t *tiley,
                        int64_t ntiles, int nyb, const int32_t *yrows, const int32_t *perm, const T *S,
                        int64_t ldS, int64_t nsrows, int64_t nkeys, int64_t n_out, T coef, T *out, int64_t ldi,
                        hipStream_t s, const int *gate) {
  typedef S2dCfg<T> C;
  const int mode = g_s2_dual.load(std::memory_order_relaxed);
  if (mode == 0 || ntiles <= 0 || nyb <= 0) return false;
  if (((uintptr_t)F1 & 15) != 0 || (ld1 * (int64_t)sizeof(T)) % 16 != 0 || nkeys % C::VEC != 0) return false;
  const int64_t nxb = ntiles / nyb;
  const int64_t ndx = ceil_div(nxb, (int64_t)C::SX), ndy = ceil_div((int64_t)nyb, (int64_t)C::SY);
  if (mode < 0 && (double)n_out > 700.0 * (double)(ndx * ndy)) return false;
  const int64_t nreg = ceil_div(ndx, (int64_t)C::RX) * ceil_div(ndy, (int64_t)C::RY);
  const int64_t nwg = ceil_div(nreg, (int64_t)8) * 8 * C::RX * C::RY;
  GVT_REQUIRE(nwg < ((int64_t)1 << 31) && nxb < ((int64_t)1 << 30), GVT_ERR_ARG, "too many stage-2 tiles");
  (void)nsrows;
  stage2_dual_kernel<T><<<(unsigned)nwg, C::NT, 0, s>>>(F1, ld1, nx, tileoff, tiley, (int)nxb, nyb, yrows, perm,
                                                        S, ldS, nsrows, nkeys, coef, out, ldi, gate);
  return true;
}

template <class T>
void launch_stage2y(const T *F1, int64_t ld1, const int64_t *tileoff, const int32_t *tilex,
                    const int32_t *tilemax, const uint8_t *grow, int64_t ntiles, int nxb,
                    const int32_t *xrows, const int32_t *perm, const T *S, int64_t ldS, int64_t nsr,
                    int64_t nkeys, int R, T coef, T *out, int64_t ldi, int64_t ldr, hipStream_t s,
                    const int *gate) {
  if (ntiles <= 0) return;
  dim3 grid((unsigned)ntiles);
  switch (R) {
    case 4:
      if (stage2y_use_pipelined())
        stage2y_pipelined_kernel<T><<<grid, kStage2Rows * 16, 0, s>>>(F1, ld1, tileoff, tilex, tilemax, grow, xrows, perm, nxb, S, ldS, nsr, nkeys, coef, out, ldi, ldr, gate);
      else
        stage2y_kernel<T, 4><<<grid, kStage2Rows * 16, 0, s>>>(F1, ld1, tileoff, tilex, tilemax, grow, xrows, perm, nxb, S, ldS, nsr, nkeys, coef, out, ldi, ldr, gate);
      break;
    case 8: stage2y_kernel<T, 8><<<grid, kStage2Rows * 16, 0, s>>>(F1, ld1, tileoff, tilex, tilemax, grow, xrows, perm, nxb, S, ldS, nsr, nkeys, coef, out, ldi, ldr, gate); break;
    default: throw Error{GVT_ERR_ARG, "internal: S-row grouped stage 2 needs a block of 4 or 8 RHS"};
  }
}

template <class T>
void launch_gemv(const T *F, int64_t ldf, int64_t nrows, int64_t ncols, bool sq, const T *sv, int R,
                 T *g, hipStream_t s) {
  if (nrows <= 0) return;
  dim3 grid((unsigned)ceil_div(nrows, 4));
  if (sq) gemv_kernel<T, true><<<grid, 256, 0, s>>>(F, ldf, nrows, ncols, sv, R, g);
  else gemv_kernel<T, false><<<grid, 256, 0, s>>>(F, ldf, nrows, ncols, sv, R, g);
}

template <class T>
void launch_gather_rows(const T *g, const int32_t *sel, int64_t n, int R, T *t, hipStream_t s) {
  if (n <= 0) return;
  gather_rows_kernel<T><<<grid1(n, 256), 256, 0, s>>>(g, sel, n, R, t);
}

template <class T>
void launch_match(const T *F, int64_t ldf, int64_t ncols, const int32_t *xsel, const int32_t *ksel,
                  int64_t n, const int32_t *operm, const int64_t *xoff, int64_t nxrows,
                  const int64_t *seg, const int32_t *other, const T *vs, int64_t nkeys, int R, T *t,
                  hipStream_t s) {
  if (n <= 0) return;
  const size_t row_bytes = (size_t)ncols * sizeof(T);
  if (operm && xoff && nxrows > 0 && row_bytes <= (64 << 10)) {
    const unsigned g = (unsigned)nxrows;
    const size_t sh = row_bytes ? row_bytes : sizeof(T);
    switch (R) {
      case 1: match_row_kernel<T, 1><<<g, 256, sh, s>>>(F, ldf, ncols, operm, xoff, ksel, seg, other, vs, nkeys, t); return;
      case 2: match_row_kernel<T, 2><<<g, 256, sh, s>>>(F, ldf, ncols, operm, xoff, ksel, seg, other, vs, nkeys, t); return;
      case 4: match_row_kernel<T, 4><<<g, 256, sh, s>>>(F, ldf, ncols, operm, xoff, ksel, seg, other, vs, nkeys, t); return;
      case 8: match_row_kernel<T, 8><<<g, 256, sh, s>>>(F, ldf, ncols, operm, xoff, ksel, seg, other, vs, nkeys, t); return;
      default: break;
    }
  }
  match_kernel<T><<<grid1(n * 16, 256), 256, 0, s>>>(F, ldf, xsel, ksel, n, seg, other, vs, nkeys, R, t);
}

template <class T>
void launch_transpose(const T *F, int64_t ldf, int64_t rows, int64_t cols, T *Ft, int64_t ldt,
                      hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
  transpose_kernel<T><<<grid, 256, 0, s>>>(F, ldf, rows, cols, Ft, ldt);
}

template <class T>
void launch_combine(const CombineArgs<T> &a, int64_t n, int R, T *U, int64_t ldu,
                    int64_t block_stride, hipStream_t s) {
  if (n <= 0) return;
  combine_kernel<T><<<grid1(n, 256), 256, 0, s>>>(a, n, R, U, ldu, block_stride);
}

template <class T>
void launch_fill(T *U, int64_t rows, int64_t cols, int64_t ld, T val, hipStream_t s) {
  if (rows * cols <= 0) return;
  fill_kernel<T><<<grid1(rows * cols, 256), 256, 0, s>>>(U, rows, cols, ld, val);
}

int64_t group_pack_blocks(int64_t n_in) { return ceil_div(n_in, kGroupPackBlock); }

template <class T>
int64_t group_stage1_setup(GroupDesc<T> &d, int64_t row0) {
  // the slice walk where the slice fits and the problem has pairs enough to
  // pay for copying it (at least 8 per F2 column); about 12 500 pairs per
  // workgroup, as many as the single product's workgroups walk on the ridge
  // workload
  d.slice = 0;
  d.nkr = d.kpr = 0;
  if (row0 >= 0 && stage1_use_slice() && d.nrows >= S1SliceCfg<T>::RB && d.nother >= 1 &&
      d.nother <= kS1SliceMaxCols && d.n_in >= 8 * d.nother && d.nkeys > 0) {
    d.slice = 1;
    d.row0 = row0;
    const int64_t nkr = std::max<int64_t>(1, std::min(ceil_div(d.n_in, (int64_t)12500), ceil_div(d.nkeys, (int64_t)64)));
    d.kpr = ceil_div(d.nkeys, nkr);
    d.nkr = ceil_div(d.nkeys, d.kpr);
    d.nkb = 0;
    return d.nkr * ceil_div(d.nrows, (int64_t)S1SliceCfg<T>::RB);
  }
  const bool wide = row0 >= 0 && stage1_use_wide() && d.nrows >= S1WideCfg<T, 1, 1>::VPL;
  d.row0 = wide ? row0 : -1;
  d.nkb = ceil_div(d.nkeys, wide ? S1WideCfg<T, 1, 1>::KB : S1Cfg<T, 1>::KB);
  return d.nkb * ceil_div(d.nrows, wide ? S1WideCfg<T, 1, 1>::ROWS : 64);
}

template <class T>
void launch_group_pack(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                       int64_t r0, const uint8_t *active, hipStream_t s) {
  if (nitems <= 0) return;
  group_pack_kernel<T><<<(unsigned)nitems, kGroupPackBlock, 0, s>>>(desc, items, R, r0, active);
}

template <class T>
void launch_group_stage1(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                         const uint8_t *active, hipStream_t s) {
  if (nitems <= 0) return;
  const unsigned g = (unsigned)nitems;
  switch (R) {
    case 1: group_stage1_kernel<T, 1><<<g, 256, 0, s>>>(desc, items, active); break;
    case 2: group_stage1_kernel<T, 2><<<g, 256, 0, s>>>(desc, items, active); break;
    case 4: group_stage1_kernel<T, 4><<<g, 256, 0, s>>>(desc, items, active); break;
    case 8: group_stage1_kernel<T, 8><<<g, 256, 0, s>>>(desc, items, active); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in grouped stage 1"};
  }
}

template <class T, int R>
static void group_slice_r(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems,
                          const uint8_t *active, size_t lds, hipStream_t s) {
  static std::once_flag once;
  std::call_once(once, [] {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&group_stage1_slice_kernel<T, R>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kS1SliceMaxCols * 256)) != hipSuccess)
      (void)hipGetLastError();
  });
  group_stage1_slice_kernel<T, R><<<(unsigned)nitems, S1SliceCfg<T>::NT, lds, s>>>(desc, items, active);
}

template <class T>
void launch_group_stage1_slice(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                               const uint8_t *active, size_t lds, hipStream_t s) {
  if (nitems <= 0) return;
  GVT_REQUIRE(lds <= (size_t)kS1SliceMaxCols * 256, GVT_ERR_ARG, "internal: slice larger than LDS");
  switch (R) {
    case 1: group_slice_r<T, 1>(desc, items, nitems, active, lds, s); break;
    case 2: group_slice_r<T, 2>(desc, items, nitems, active, lds, s); break;
    case 4: group_slice_r<T, 4>(desc, items, nitems, active, lds, s); break;
    case 8: group_slice_r<T, 8>(desc, items, nitems, active, lds, s); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in grouped stage 1"};
  }
}

template <class T>
void launch_group_stage2(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                         int64_t r0, const uint8_t *active, hipStream_t s) {
  if (nitems <= 0) return;
  const unsigned g = (unsigned)nitems;
  const int nt = S2Cfg<T, 1>::NT;
  // items: the tiles of R's class (F1-row groups for 1-2 RHS, S-row groups for 4-8)
  switch (R) {
    case 1: group_stage2_kernel<T, 1><<<g, nt, 0, s>>>(desc, items, r0, active); break;
    case 2: group_stage2_kernel<T, 2><<<g, nt, 0, s>>>(desc, items, r0, active); break;
    case 4:
      if (stage2y_use_pipelined())
        group_stage2y_pipelined_kernel<T><<<g, kStage2Rows * 16, 0, s>>>(desc, items, r0, active);
      else
        group_stage2y_kernel<T, 4><<<g, kStage2Rows * 16, 0, s>>>(desc, items, r0, active);
      break;
    case 8: group_stage2y_kernel<T, 8><<<g, kStage2Rows * 16, 0, s>>>(desc, items, r0, active); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in grouped stage 2"};
  }
}

#define GVT_INSTANTIATE(T)                                                                      \
  template void launch_pack_v<T>(const T *, int64_t, const int32_t *, int64_t, int, T *,          \
                                 hipStream_t, const int *);                                      \
  template void launch_segsum<T>(const int64_t *, const T *, int64_t, int, T *, hipStream_t);    \
  template int64_t group_stage1_setup<T>(GroupDesc<T> &, int64_t);                               \
  template void launch_group_stage1_slice<T>(const GroupDesc<T> *, const GroupItem *, int64_t, int, \
                                             const uint8_t *, size_t, hipStream_t);               \
  template void launch_stage1<T>(const T *, int64_t, const int32_t *, int64_t, int64_t,         \
                                 const int64_t *, const int32_t *, int64_t, const T *, int64_t,  \
                                 int, T *, int64_t, hipStream_t, const int *);\
  template void launch_colscale<T>(const T *, int64_t, const int32_t *, int64_t, const T *,      \
                                   int64_t, int, T *, int64_t, hipStream_t);                     \
  template void launch_stage2<T>(const T *, int64_t, int64_t, const int64_t *, const int32_t *,  \
                                 const int32_t *, const uint8_t *, int64_t, int, const int32_t *,\
                                 const int32_t *,                                                \
                                 const T *, int64_t, int64_t, int64_t, int, T, T *, int64_t,     \
                                 int64_t, hipStream_t, const int *);                             \
  template bool launch_stage2_dual<T>(const T *, int64_t, int64_t, const int64_t *, const int32_t *, \
                                      int64_t, int, const int32_t *, const int32_t *, const T *,   \
                                      int64_t, int64_t, int64_t, int64_t, T, T *, int64_t,         \
                                      hipStream_t, const int *);                                    \
  template void launch_stage2y<T>(const T *, int64_t, const int64_t *, const int32_t *,          \
                                  const int32_t *, const uint8_t *, int64_t, int,                 \
                                  const int32_t *, const int32_t *,                               \
                                  const T *, int64_t, int64_t, int64_t, int, T, T *, int64_t,     \
                                  int64_t, hipStream_t, const int *);                             \
  template void launch_gemv<T>(const T *, int64_t, int64_t, int64_t, bool, const T *, int, T *,  \
                               hipStream_t);                                                     \
  template void launch_gather_rows<T>(const T *, const int32_t *, int64_t, int, T *,             \
                                      hipStream_t);                                              \
  template void launch_match<T>(const T *, int64_t, int64_t, const int32_t *, const int32_t *,   \
                                int64_t, const int32_t *, const int64_t *, int64_t,              \
                                const int64_t *, const int32_t *, const T *, int64_t, int, T *,  \
                                hipStream_t);                                                    \
  template void launch_transpose<T>(const T *, int64_t, int64_t, int64_t, T *, int64_t,          \
                                    hipStream_t);                                                \
  template void launch_combine<T>(const CombineArgs<T> &, int64_t, int, T *, int64_t, int64_t,   \
                                  hipStream_t);                                                  \
  template void launch_fill<T>(T *, int64_t, int64_t, int64_t, T, hipStream_t);                 \
  template void launch_group_pack<T>(const GroupDesc<T> *, const GroupItem *, int64_t, int,      \
                                     int64_t, const uint8_t *, hipStream_t);                     \
  template void launch_group_stage1<T>(const GroupDesc<T> *, const GroupItem *, int64_t, int,    \
                                       const uint8_t *, hipStream_t);                            \
  template void launch_group_stage2<T>(const GroupDesc<T> *, const GroupItem *, int64_t, int,    \
                                       int64_t, const uint8_t *, hipStream_t);

GVT_INSTANTIATE(double)
GVT_INSTANTIATE(float)

}  // namespace gvt
