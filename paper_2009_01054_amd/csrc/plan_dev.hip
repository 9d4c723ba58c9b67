// Device-side plan construction: index validation and unique marks (Table 1),
// the input pairs sorted into stage-1 key segments, output groupings for the
// Cartesian match terms and the stage-2 tile orders of Theorem 1's two
// stages.  Sorts are stable LSD radix sorts over the packed keys, so each
// array equals the one a stable host counting sort gives.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cstdlib>

#include "kernels.h"
#include "plan_dev.h"

namespace gvt {

namespace {

constexpr int PB = 256;  // threads per block of the plan kernels

inline unsigned grid_for(int64_t n) {
  const int64_t b = ceil_div(n > 0 ? n : 1, PB);
  return (unsigned)(b < 65535 * 16 ? b : 65535 * 16);
}

void *scratch_get(DevScratch &sc, size_t bytes, hipStream_t s) {
  if (bytes > sc.mem.bytes && sc.mem.p) {
    // the old buffer may still be read by kernels queued on s
    GVT_HIP_CHECK(hipStreamSynchronize(s));
  }
  return sc.mem.ensure(bytes);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---- probe ------------------------------------------------------------------
struct ProbeArgs {
  const int32_t *x[4];
  int64_t n[4];
  int64_t lim[4];
  uint8_t *seen[4];
  int64_t div[4][2];  // natural-order check: x[j] == j / div (even arrays) or j % div (odd); 0 = none
};

__global__ __launch_bounds__(PB) void probe_kernel(ProbeArgs a, unsigned long long *bad, int *notnat) {
  const int y = blockIdx.y;
  const int32_t *x = a.x[y];
  const int64_t n = a.n[y], lim = a.lim[y];
  uint8_t *seen = a.seen[y];
  int mism = 0;
  for (int64_t j = (int64_t)blockIdx.x * PB + threadIdx.x; j < n; j += (int64_t)gridDim.x * PB) {
    const int32_t v = x[j];
    if (v < 0 || v >= lim) {
      atomicMin(bad + y, (unsigned long long)j);
    } else {
      seen[v] = 1;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t d = a.div[y][q];
      if (d > 0) mism |= (int64_t)v != ((y & 1) ? j % d : j / d);
    }
  }
  if (mism) *notnat = 1;
}

// ---- sorting -----------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs by the low nbits bits of the key,
// in passes of digits of at most kRsMaxW bits (the key width split evenly).  A
// pass is three launches with no waiting between workgroups:
//   count:   per tile of kRsTile pairs, the count of each digit value;
//   tscan:   per digit value (one wave each), the exclusive prefix of its
//            counts over the tiles, in place, and its total;
//   scatter: per tile, every pair goes to base(digit) + prefix(digit, tile) +
//            the pairs of the same digit before it in the tile, where base is
//            the exclusive prefix of the totals (scanned by each block).
// The scatter walks its tile in rounds of kRsT pairs; within a round a pair's
// rank among its wave's pairs of the same digit comes from ballots on the digit
// bits, and the counts of the waves before it from per-wave counts in LDS
// tagged with the round; after the round each (digit, wave) leader adds its
// count to the digit's running position (integer LDS atomics).  Pairs keep their order within a digit in every pass,
// so the result is the unique stable order, as a library sort's.
constexpr int kRsT = 256;                 // threads per block
constexpr int kRsRounds = 4;  // rounds of kRsT pairs per tile (ridge plans: 0.187 ms, 0.194 with 2, 0.206 with 8)
constexpr int kRsTile = kRsT * kRsRounds;
constexpr int kRsMaxW = 10;               // widest digit
constexpr int kRsMaxB = 1 << kRsMaxW;

template <class K>
__global__ __launch_bounds__(kRsT) void rs_count_kernel(const K *__restrict__ key, int64_t n, int sh, int width,
                                                        int64_t nt, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t h[kRsMaxB];
  const int nb = 1 << width;
  for (int b = threadIdx.x; b < nb; b += kRsT) h[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int j = 0; j < kRsRounds; ++j) {
    const int64_t p = base + (int64_t)j * kRsT + threadIdx.x;
    if (p < n) atomicAdd(&h[(int)((key[p] >> sh) & (K)(nb - 1))], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += kRsT) cnt[(int64_t)b * nt + blockIdx.x] = h[b];
}

// one wave per digit value: 64 tiles' counts per step, scanned across the wave
__global__ __launch_bounds__(kRsT) void rs_tscan_kernel(uint32_t *__restrict__ cnt, int64_t nt, int nb,
                                                        uint32_t *__restrict__ total) {
  const int b = blockIdx.x * (kRsT / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (b >= nb) return;  // wave-uniform
  uint32_t *c = cnt + (int64_t)b * nt;
  uint32_t carry = 0;
  for (int64_t t0 = 0; t0 < nt; t0 += 64) {
    const int64_t t = t0 + lane;
    const uint32_t e = t < nt ? c[t] : 0u;
    uint32_t x = e;  // inclusive prefix over the wave
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (t < nt) c[t] = carry + x - e;
    carry += __shfl(x, 63, 64);
  }
  if (lane == 0) total[b] = carry;
}

template <class K>
__global__ __launch_bounds__(kRsT) void rs_scatter_kernel(const K *__restrict__ kin, const int32_t *__restrict__ vin,
                                                          K *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
                                                          int sh, int width, int64_t nt,
                                                          const uint32_t *__restrict__ cnt,
                                                          const uint32_t *__restrict__ total) {
  constexpr int NW = kRsT / 64;
  __shared__ uint32_t run[kRsMaxB];
  __shared__ uint32_t wc[NW][kRsMaxB];  // (round + 1) << 8 | the wave's count of a digit
  __shared__ uint32_t part[kRsT];
  const int nb = 1 << width;
  const int per = nb / kRsT > 0 ? nb / kRsT : 1;  // digits per thread in the base scan
  // base(digit): exclusive prefix of the totals; each thread sums `per` digits
  uint32_t s = 0;
  const int b0 = threadIdx.x * per;
  for (int b = b0; b < b0 + per && b < nb; ++b) s += total[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kRsT; o <<= 1) {
    const uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t acc = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int b = b0; b < b0 + per && b < nb; ++b) {
    run[b] = acc + cnt[(int64_t)b * nt + blockIdx.x];
    acc += total[b];
  }
  for (int i = threadIdx.x; i < NW * kRsMaxB; i += kRsT) (&wc[0][0])[i] = 0;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const unsigned long long below = (1ull << lane) - 1;
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int j = 0; j < kRsRounds; ++j) {
    const int64_t p = base + (int64_t)j * kRsT + threadIdx.x;
    const bool valid = p < n;
    const K k = valid ? kin[p] : K(0);
    const int32_t v = valid ? vin[p] : 0;
    const int d = valid ? (int)((k >> sh) & (K)(nb - 1)) : nb;  // nb: past the end
    // the lanes of this wave whose pairs have the same digit (and validity)
    unsigned long long same = ~0ull;
    for (int bit = 0; bit <= width; ++bit) {
      const unsigned long long bl = __ballot((d >> bit) & 1);
      same &= ((d >> bit) & 1) ? bl : ~bl;
    }
    const int rank = __popcll(same & below);
    const uint32_t tag = (uint32_t)(j + 1) << 8;
    __syncthreads();  // the previous round's readers of run and wc are done
    if (valid && rank == 0) wc[w][d] = tag | (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + (uint32_t)rank;
      for (int w2 = 0; w2 < w; ++w2) {
        const uint32_t e = wc[w2][d];
        if ((e & ~0xffu) == tag) pos += e & 0xffu;
      }
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();  // every position of the round is taken
    // each (digit, wave) leader moves its digit's running position past its pairs
    if (valid && rank == 0) atomicAdd(&run[d], (uint32_t)__popcll(same));
  }
}

// GVT_PLAN_LIBRARY_SORT=1: the library's radix sort (hipCUB) instead, for comparison
bool use_library_sort() {
  const char *e = std::getenv("GVT_PLAN_LIBRARY_SORT");
  return e && std::atoi(e) != 0;
}

template <class K>
size_t library_sort_bytes(int64_t n) {
  size_t b = 0;
  GVT_HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const K *)nullptr, (K *)nullptr,
                                                   (const int32_t *)nullptr, (int32_t *)nullptr,
                                                   (int)n, 0, (int)(8 * sizeof(K)), (hipStream_t)0));
  return b;
}

template <class K>
size_t radix_sort_bytes(int64_t n) {
  const int64_t nt = ceil_div(n > 0 ? n : 1, kRsTile);
  return align256(n * sizeof(K)) + align256(n * sizeof(int32_t)) + align256((size_t)kRsMaxB * nt * 4) +
         align256((size_t)kRsMaxB * 4);
}

template <class K>
size_t sort_temp_bytes(int64_t n) {
  return std::max(radix_sort_bytes<K>(n), library_sort_bytes<K>(n));
}

template <class K>
void radix_sort_pairs(const K *kin, K *kout, const int32_t *vin, int32_t *vout, int64_t n, int nbits, void *temp,
                      hipStream_t s) {
  GVT_REQUIRE(n < ((int64_t)1 << 31), GVT_ERR_ARG, "internal: sort of 2^31 pairs or more");
  const int64_t nt = ceil_div(n, kRsTile);
  char *t = static_cast<char *>(temp);
  K *ktmp = reinterpret_cast<K *>(t);
  int32_t *vtmp = reinterpret_cast<int32_t *>(t + align256(n * sizeof(K)));
  uint32_t *cnt = reinterpret_cast<uint32_t *>(t + align256(n * sizeof(K)) + align256(n * 4));
  uint32_t *total = cnt + align256((size_t)kRsMaxB * nt * 4) / 4;
  const int bits = nbits > 0 ? nbits : 1;
  const int passes = (bits + kRsMaxW - 1) / kRsMaxW;
  const int width = (bits + passes - 1) / passes;
  const K *ks = kin;
  const int32_t *vs = vin;
  for (int q = 0; q < passes; ++q) {
    const int sh = q * width, wq = std::min(width, bits - sh);
    // the last pass writes the output; the passes alternate between it and the temporaries
    const bool to_out = (passes - 1 - q) % 2 == 0;
    K *kd = to_out ? kout : ktmp;
    int32_t *vd = to_out ? vout : vtmp;
    rs_count_kernel<K><<<(unsigned)nt, kRsT, 0, s>>>(ks, n, sh, wq, nt, cnt);
    rs_tscan_kernel<<<(unsigned)ceil_div(1 << wq, kRsT / 64), kRsT, 0, s>>>(cnt, nt, 1 << wq, total);
    rs_scatter_kernel<K><<<(unsigned)nt, kRsT, 0, s>>>(ks, vs, kd, vd, n, sh, wq, nt, cnt, total);
    ks = kd;
    vs = vd;
  }
  check_launch(s);
}

template <class K>
void sort_pairs(const K *kin, K *kout, const int32_t *vin, int32_t *vout, int64_t n, int nbits,
                void *temp, size_t temp_bytes, hipStream_t s) {
  if (n <= 0) return;
  if (use_library_sort()) {
    size_t tb = temp_bytes;
    GVT_HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(temp, tb, kin, kout, vin, vout, (int)n, 0,
                                                     nbits > 0 ? nbits : 1, s));
    return;
  }
  radix_sort_pairs<K>(kin, kout, vin, vout, n, nbits, temp, s);
}

__global__ void iota_kernel(int32_t *v, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * PB + threadIdx.x; j < n; j += (int64_t)gridDim.x * PB)
    v[j] = (int32_t)j;
}

// start[k] = first position p of sorted keys whose bucket (key >> sh) is >= k,
// k in [0, nb]; every k is written by exactly one position p in [0, n].
template <class K>
__global__ void bucket_starts_kernel(const K *__restrict__ key, int64_t n, int sh, int64_t nb,
                                     int64_t *__restrict__ start) {
  for (int64_t p = (int64_t)blockIdx.x * PB + threadIdx.x; p <= n; p += (int64_t)gridDim.x * PB) {
    const int64_t kprev = p == 0 ? -1 : (int64_t)(key[p - 1] >> sh);
    const int64_t kcur = p == n ? nb : (int64_t)(key[p] >> sh);
    for (int64_t k = kprev + 1; k <= kcur; ++k) start[k] = p;
  }
}

// ---- input sort -------------------------------------------------------------------
template <class K>
__global__ void pair_keys_kernel(const int32_t *__restrict__ key, const int32_t *__restrict__ other,
                                 int64_t n, int ob, K *__restrict__ ck, int32_t *__restrict__ val) {
  for (int64_t j = (int64_t)blockIdx.x * PB + threadIdx.x; j < n; j += (int64_t)gridDim.x * PB) {
    ck[j] = ((K)(uint32_t)key[j] << ob) | (K)(uint32_t)other[j];
    val[j] = (int32_t)j;
  }
}

template <class K>
__global__ void split_other_kernel(const K *__restrict__ ck, int64_t n, int ob,
                                   int32_t *__restrict__ other) {
  const K mask = ob > 0 ? (((K)1 << ob) - 1) : (K)0;
  for (int64_t p = (int64_t)blockIdx.x * PB + threadIdx.x; p < n; p += (int64_t)gridDim.x * PB)
    other[p] = (int32_t)(ck[p] & mask);
}

template <class K> size_t input_sort_bytes(int64_t n) {
  return 2 * align256(n * sizeof(K)) + align256(n * sizeof(int32_t)) + sort_temp_bytes<K>(n);
}

template <class K>
void input_sort_t(const int32_t *key, int64_t nkeys, const int32_t *other, int64_t nother, int64_t n,
                  int32_t *perm, int32_t *other_out, int64_t *seg, DevScratch &sc, hipStream_t s) {
  const int ob = bits_for(nother), kb = bits_for(nkeys);
  const size_t tb = sort_temp_bytes<K>(n);
  const size_t o_kout = align256(n * sizeof(K)), o_val = o_kout + align256(n * sizeof(K));
  const size_t o_tmp = o_val + align256(n * sizeof(int32_t));
  char *base = static_cast<char *>(scratch_get(sc, o_tmp + tb, s));
  K *kin = reinterpret_cast<K *>(base);
  K *kout = reinterpret_cast<K *>(base + o_kout);
  int32_t *val = reinterpret_cast<int32_t *>(base + o_val);
  pair_keys_kernel<K><<<grid_for(n), PB, 0, s>>>(key, other, n, ob, kin, val);
  sort_pairs<K>(kin, kout, val, perm, n, ob + kb, base + o_tmp, tb, s);
  split_other_kernel<K><<<grid_for(n), PB, 0, s>>>(kout, n, ob, other_out);
  bucket_starts_kernel<K><<<grid_for(n + 1), PB, 0, s>>>(kout, n, ob, nkeys, seg);
  check_launch(s);
}

// ---- stage-2 tiles ---------------------------------------------------------------
__global__ void tile_keys_kernel(const int32_t *__restrict__ gx, const int32_t *__restrict__ sy,
                                 const int32_t *__restrict__ rowmap, int64_t n, TileDims td,
                                 uint32_t *__restrict__ tkey, int32_t *__restrict__ stg,
                                 int32_t *__restrict__ val) {
  for (int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x; i < n; i += (int64_t)gridDim.x * PB) {
    const int64_t yr = rowmap[sy[i]], xv = gx[i];
    const int64_t grp = td.swap ? yr : xv, st = td.swap ? xv : yr;
    const int64_t tile = (grp / td.rows_per_tile) * td.nsb + st / td.sbs;
    tkey[i] = (uint32_t)(tile * td.rows_per_tile + grp % td.rows_per_tile);
    stg[i] = (int32_t)st;
    val[i] = (int32_t)i;
  }
}

__global__ void invert_kernel(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ inv) {
  for (int64_t p = (int64_t)blockIdx.x * PB + threadIdx.x; p < n; p += (int64_t)gridDim.x * PB)
    inv[perm[p]] = (int32_t)p;
}

__global__ void gather_kernel(const int32_t *__restrict__ src, const int32_t *__restrict__ idx,
                              int64_t n, int32_t *__restrict__ dst) {
  for (int64_t q = (int64_t)blockIdx.x * PB + threadIdx.x; q < n; q += (int64_t)gridDim.x * PB)
    dst[q] = src[idx[q]];
}

// Group order of each tile: 32 lanes per tile (two tiles per wave), lane g
// holds row g's output count and finds its rank among the tile's rows by
// descending count, ties by row, by reading the other counts across lanes.
__global__ void tile_order_kernel(const int64_t *__restrict__ sgk, int64_t ntiles,
                                  uint8_t *__restrict__ grow) {
  static_assert(kStage2Rows == 32 && PB % 64 == 0, "two tiles per wave");
  const int lane = threadIdx.x & 63, g = lane & 31, half = lane & 32;
  const int64_t t = ((int64_t)blockIdx.x * PB + threadIdx.x) / kStage2Rows;
  const bool live = t < ntiles;
  const int c = live ? (int)(sgk[t * kStage2Rows + g + 1] - sgk[t * kStage2Rows + g]) : 0;
  int rank = 0;
  for (int h = 0; h < kStage2Rows; ++h) {
    const int ch = __shfl(c, half | h, 64);
    rank += ch > c || (ch == c && h < g);
  }
  if (live) grow[t * kStage2Rows + rank] = (uint8_t)g;
}

__global__ void tile_meta_kernel(const int64_t *__restrict__ sgk, TileDims td,
                                 int64_t *__restrict__ toff, int32_t *__restrict__ tiley,
                                 int32_t *__restrict__ tilemax) {
  constexpr int R = kStage2Rows;  // the caller checks td.rows_per_tile
  for (int64_t t = (int64_t)blockIdx.x * PB + threadIdx.x; t < td.ntiles;
       t += (int64_t)gridDim.x * PB) {
    int64_t b[R + 1];  // the tile's group starts, all loads in flight together
#pragma unroll
    for (int g = 0; g <= R; ++g) b[g] = sgk[t * R + g];
    int32_t mx = 0;
#pragma unroll
    for (int g = 0; g <= R; ++g) {
      toff[t * (R + 1) + g] = b[g];
      if (g < R) {
        const int64_t c = b[g + 1] - b[g];
        mx = c > mx ? (int32_t)c : mx;
      }
    }
    tilemax[t] = mx;
    const int64_t sbk = t % td.nsb, y0 = sbk * td.sbs;
    const int64_t cnt = td.nstg_rows - y0 < td.sbs ? td.nstg_rows - y0 : td.sbs;
    tiley[2 * t] = (int32_t)(y0 < td.nstg_rows ? y0 : td.nstg_rows);
    tiley[2 * t + 1] = (int32_t)(cnt > 0 ? cnt : 0);
  }
}

}  // namespace

void dev_probe(const int32_t *const *x, const int64_t *n, const int64_t *lim, const int64_t *range,
               int narr, int64_t nat_out_cols, int64_t nat_in_cols, DevScratch &sc,
               ProbeResult &res, hipStream_t s) {
  ProbeArgs a{};
  size_t off = 64;  // bad[4] (u64) + notnat (int), padded
  size_t soff[4] = {0, 0, 0, 0};
  int64_t nmax = 0;
  for (int i = 0; i < narr; ++i) {
    a.x[i] = x[i];
    a.n[i] = n[i];
    a.lim[i] = lim[i];
    soff[i] = off;
    off += align256((size_t)std::max<int64_t>(range[i], 1));
    nmax = std::max(nmax, n[i]);
    // arrays 0/1 (output a, b) and 2/3 (input c, e); with two arrays the
    // output pairs are the input pairs and carry both checks
    const int64_t own = i < 2 ? nat_out_cols : nat_in_cols;
    a.div[i][0] = own;
    a.div[i][1] = (narr == 2) ? nat_in_cols : 0;
  }
  const size_t total = off;
  char *base = static_cast<char *>(scratch_get(sc, total, s));
  for (int i = 0; i < narr; ++i) a.seen[i] = reinterpret_cast<uint8_t *>(base + soff[i]);
  GVT_HIP_CHECK(hipMemsetAsync(base, 0, total, s));
  GVT_HIP_CHECK(hipMemsetAsync(base, 0xff, 32, s));
  if (nmax > 0) {
    const dim3 grid(std::min<unsigned>(grid_for(nmax), 2048u), (unsigned)narr);
    probe_kernel<<<grid, PB, 0, s>>>(a, reinterpret_cast<unsigned long long *>(base),
                                     reinterpret_cast<int *>(base + 32));
    check_launch(s);
  }
  std::vector<uint8_t> h(total);
  GVT_HIP_CHECK(hipMemcpyAsync(h.data(), base, total, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < 4; ++i) res.bad[i] = -1;
  for (int i = 0; i < narr; ++i) {
    unsigned long long b;
    std::memcpy(&b, h.data() + 8 * i, 8);
    res.bad[i] = b == ULLONG_MAX ? -1 : (int64_t)b;
    res.seen[i].assign(h.data() + soff[i], h.data() + soff[i] + range[i]);
  }
  int notnat;
  std::memcpy(&notnat, h.data() + 32, 4);
  res.nat = (nat_out_cols > 0 || nat_in_cols > 0) && notnat == 0;
}

size_t dev_input_sort_bytes(int64_t nkeys, int64_t nother, int64_t n) {
  return bits_for(nkeys) + bits_for(nother) <= 32 ? input_sort_bytes<uint32_t>(n)
                                                  : input_sort_bytes<uint64_t>(n);
}

size_t dev_group_rows_bytes(int64_t n) { return 2 * align256(n * 4) + sort_temp_bytes<uint32_t>(n); }

size_t dev_tiles_bytes(int64_t n, int64_t nbuckets) {
  return 4 * align256(n * 4) + align256((nbuckets + 1) * 8) + sort_temp_bytes<uint32_t>(n);
}

void dev_reserve(DevScratch &sc, size_t bytes, hipStream_t s) { (void)scratch_get(sc, bytes, s); }

void dev_input_sort(const int32_t *key, int64_t nkeys, const int32_t *other, int64_t nother,
                    int64_t n, int32_t *perm, int32_t *other_out, int64_t *seg, DevScratch &sc,
                    hipStream_t s) {
  if (bits_for(nkeys) + bits_for(nother) <= 32)
    input_sort_t<uint32_t>(key, nkeys, other, nother, n, perm, other_out, seg, sc, s);
  else
    input_sort_t<uint64_t>(key, nkeys, other, nother, n, perm, other_out, seg, sc, s);
}

void dev_invert(const int32_t *perm, int64_t n, int32_t *inv, hipStream_t s) {
  if (n <= 0) return;
  invert_kernel<<<grid_for(n), PB, 0, s>>>(perm, n, inv);
  check_launch(s);
}

void dev_group_rows(const int32_t *row, int64_t nrows, int64_t n, int32_t *perm, int64_t *off,
                    DevScratch &sc, hipStream_t s) {
  const size_t tb = sort_temp_bytes<uint32_t>(n);
  const size_t o_val = align256(n * 4), o_tmp = o_val + align256(n * 4);
  char *base = static_cast<char *>(scratch_get(sc, o_tmp + tb, s));
  uint32_t *kout = reinterpret_cast<uint32_t *>(base);
  int32_t *val = reinterpret_cast<int32_t *>(base + o_val);
  iota_kernel<<<grid_for(n), PB, 0, s>>>(val, n);
  sort_pairs<uint32_t>(reinterpret_cast<const uint32_t *>(row), kout, val, perm, n, bits_for(nrows),
                       base + o_tmp, tb, s);
  bucket_starts_kernel<uint32_t><<<grid_for(n + 1), PB, 0, s>>>(kout, n, 0, nrows, off);
  check_launch(s);
}

void dev_tiles(const int32_t *gx, const int32_t *sy, const int32_t *rowmap, int64_t n,
               const TileDims &td, int32_t *perm, int32_t *yrows, int64_t *toff, int32_t *tiley,
               int32_t *tilemax, uint8_t *grow, DevScratch &sc, hipStream_t s) {
  GVT_REQUIRE(td.rows_per_tile == kStage2Rows, GVT_ERR_ARG, "internal: stage-2 tile height");
  const int64_t nb = td.ntiles * td.rows_per_tile;
  const size_t tb = sort_temp_bytes<uint32_t>(n);
  const size_t o_kout = align256(n * 4), o_stg = o_kout + align256(n * 4);
  const size_t o_val = o_stg + align256(n * 4), o_sgk = o_val + align256(n * 4);
  const size_t o_tmp = o_sgk + align256((nb + 1) * 8);
  char *base = static_cast<char *>(scratch_get(sc, o_tmp + tb, s));
  uint32_t *tkey = reinterpret_cast<uint32_t *>(base);
  uint32_t *kout = reinterpret_cast<uint32_t *>(base + o_kout);
  int32_t *stg = reinterpret_cast<int32_t *>(base + o_stg);
  int32_t *val = reinterpret_cast<int32_t *>(base + o_val);
  int64_t *sgk = reinterpret_cast<int64_t *>(base + o_sgk);
  tile_keys_kernel<<<grid_for(n), PB, 0, s>>>(gx, sy, rowmap, n, td, tkey, stg, val);
  sort_pairs<uint32_t>(tkey, kout, val, perm, n, bits_for(nb), base + o_tmp, tb, s);
  gather_kernel<<<grid_for(n), PB, 0, s>>>(stg, perm, n, yrows);
  bucket_starts_kernel<uint32_t><<<grid_for(n + 1), PB, 0, s>>>(kout, n, 0, nb, sgk);
  tile_meta_kernel<<<grid_for(td.ntiles), PB, 0, s>>>(sgk, td, toff, tiley, tilemax);
  tile_order_kernel<<<(unsigned)std::max<int64_t>(1, ceil_div(td.ntiles, PB / kStage2Rows)), PB, 0, s>>>(
      sgk, td.ntiles, grow);
  check_launch(s);
}

}  // namespace gvt
