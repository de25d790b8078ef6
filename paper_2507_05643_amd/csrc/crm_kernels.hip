// HIP kernels of the CRM particle step for gfx950 (CDNA4, wave64).
//
// Paper: arXiv 2507.05643 (Chrono::CRM). Sections cited per kernel.
// Nothing here is a dense contraction, so no MFMA: the neighbour interaction
// is FP32 VALU work over cell-sorted records, the binning/compaction steps are
// HBM streams built from wave64 ballots and block scans.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "crm_device.h"

namespace crm {
namespace {


template <typename T>
__device__ inline T wave_incl_scan(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan over the kBlock threads of a workgroup; `total` gets the sum.
template <typename T>
__device__ inline T block_excl_scan(T v, T& total) {
  __shared__ T wsum[kBlock / kWave];
  T incl = wave_incl_scan(v);
  if (lane_id() == kWave - 1) wsum[wave_id()] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / kWave; ++k) {
    T s = wsum[k];
    pre += (k < wave_id()) ? s : T(0);
    tot += s;
  }
  __syncthreads();
  total = tot;
  return pre + incl - v;
}

// ---------------------------------------------------------------- scans ---
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TIn* __restrict__ in, int64_t n,
                                                        TOut* __restrict__ bsum) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TOut acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) acc += (TOut)in[i];
  }
  TOut tot;
  block_excl_scan(acc, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// The apply pass also forms its tile's carry-in, the sum of the earlier
// tiles' totals (integers, so the order of the sum does not matter), and the
// last tile writes the grand total: two launches per scan.
template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const TIn* __restrict__ in, int64_t n,
                                                       const TOut* __restrict__ bsum, int64_t nb,
                                                       TOut* __restrict__ out, TOut* __restrict__ out_total) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TOut part = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kBlock) part += bsum[i];
  TOut carry;
  block_excl_scan(part, carry);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    TOut v = (i < n) ? (TOut)in[i] : TOut(0);
    TOut tot;
    TOut ex = block_excl_scan(v, tot);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
  if ((int64_t)blockIdx.x == nb - 1 && threadIdx.x == 0) *out_total = carry;
}

template <typename T>
__global__ void k_set_one(T* p, T v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <typename TIn, typename TOut>
hipError_t scan_impl(const TIn* in, TOut* out, int64_t n, TOut* tmp, hipStream_t s) {
  if (n <= 0) {
    k_set_one<TOut><<<1, 64, 0, s>>>(out, TOut(0));
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  k_scan_reduce<TIn, TOut><<<(unsigned)nb, kBlock, 0, s>>>(in, n, tmp);
  k_scan_apply<TIn, TOut><<<(unsigned)nb, kBlock, 0, s>>>(in, n, tmp, nb, out, out + n);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * kBlock;
  for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------- compaction ---
// Order-preserving stream compaction: per-block counts from wave ballots, an
// exclusive scan of the counts, then each lane writes at block offset + wave
// offset + popcount of the lower lanes of its ballot.
struct PredFlags {
  const uint8_t* f;
  __device__ bool operator()(int64_t i) const { return f[i] != 0; }
};
struct PredKind {
  const float4* p;
  uint32_t kind;
  __device__ bool operator()(int64_t i) const { return (__float_as_uint(p[i].w) & 3u) == kind; }
};

struct PredNonzero {
  const uint32_t* c;
  __device__ bool operator()(int64_t i) const { return c[i] != 0u; }
};

template <class Pred>
__global__ __launch_bounds__(kBlock) void k_pred_count(Pred pr, int64_t n, uint32_t* __restrict__ bcnt) {
  __shared__ uint32_t ws[kBlock / kWave];
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool p = (i < n) && pr(i);
  uint64_t m = __ballot(p);
  if (lane_id() == 0) ws[wave_id()] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kBlock / kWave; ++k) t += ws[k];
    bcnt[blockIdx.x] = t;
  }
}

template <class Pred>
__global__ __launch_bounds__(kBlock) void k_pred_write(Pred pr, int64_t n, const uint32_t* __restrict__ boff,
                                                       int32_t* __restrict__ out, uint64_t* __restrict__ count_dst) {
  // the count (the scan's total, boff[gridDim.x]) goes out with the last block
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count_dst = (uint64_t)boff[gridDim.x];
  __shared__ uint32_t ws[kBlock / kWave];
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool p = (i < n) && pr(i);
  uint64_t m = __ballot(p);
  if (lane_id() == 0) ws[wave_id()] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t pre = boff[blockIdx.x];
  for (int k = 0; k < wave_id(); ++k) pre += ws[k];
  if (p) out[pre + (uint32_t)__popcll(m & lanemask_lt())] = (int32_t)i;
}

// Compaction of the activity flags (all N particles at every activity
// rebuild): each thread takes 16 flags with one 16-byte load (the flag array is
// padded with zeros to a multiple of 16), so both passes stream the flags at
// close to HBM speed. Order-preserving: thread ranges are in index order.
constexpr int kFlagsPer = 16;
constexpr int64_t kFlagsTile = (int64_t)kBlock * kFlagsPer;

__device__ inline uint32_t flag_mask(const uint4* __restrict__ f16, int64_t chunk, int64_t nchunks) {
  if (chunk >= nchunks) return 0u;
  const uint4 v = f16[chunk];
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int b = 0; b < 4; ++b) m |= ((w[q] >> (8 * b)) & 0xffu) ? (1u << (4 * q + b)) : 0u;
  return m;
}

__global__ __launch_bounds__(kBlock) void k_flags_write(const uint4* __restrict__ f16, int64_t nchunks,
                                                        const uint32_t* __restrict__ boff, int32_t* __restrict__ out) {
  if (boff[blockIdx.x + 1] == boff[blockIdx.x]) return;   // no flagged particle in this tile
  const int64_t chunk = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t m = flag_mask(f16, chunk, nchunks);
  uint32_t tot;
  uint32_t pos = boff[blockIdx.x] + block_excl_scan((uint32_t)__popc(m), tot);
  while (m) {
    const int b = __builtin_ctz(m);
    out[pos++] = (int32_t)(chunk * kFlagsPer + b);
    m &= m - 1u;
  }
}

__global__ void k_copy2(uint64_t* dst, const uint64_t* a, const uint64_t* b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = *a;
    dst[1] = *b;
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_f64(double* __restrict__ dst, const double* __restrict__ src,
                                                     int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_store_count(uint64_t* dst, const uint32_t* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = (uint64_t)*src;
}

template <class Pred>
hipError_t compact_impl(Pred pr, int64_t n, int32_t* out, uint64_t* count_dst, uint32_t* tmp,
                        hipStream_t s) {
  if (n <= 0) {
    k_set_one<uint64_t><<<1, 64, 0, s>>>(count_dst, 0ull);
    return hipGetLastError();
  }
  const int64_t nb = (n + kBlock - 1) / kBlock;
  uint32_t* bcnt = tmp;
  uint32_t* boff = tmp + nb;
  uint32_t* stmp = boff + nb + 1;
  k_pred_count<Pred><<<(unsigned)nb, kBlock, 0, s>>>(pr, n, bcnt);
  hipError_t e = scan_impl<uint32_t, uint32_t>(bcnt, boff, nb, stmp, s);
  if (e != hipSuccess) return e;
  k_pred_write<Pred><<<(unsigned)nb, kBlock, 0, s>>>(pr, n, boff, out, count_dst);
  return hipGetLastError();
}

// ---------------------------------------------------- markers and flags ---
// A cell index clamped to a grid of dim cells (particles outside are binned
// into the edge cells).
__device__ inline int32_t clamp_cell(int32_t c, int32_t dim) { return c < 0 ? 0 : (c > dim - 1 ? dim - 1 : c); }

// The activity pass's pre-test reads its own compact copy of each particle's
// coordinates (FP32 x, y, z: 12 bytes) or cells (cell-offset positions: the
// 8 bytes of d.zw) instead of a 16-byte plane. The copy is written wherever the
// master store's positions change (the list rebuild's scatter, the markers'
// placement) and refilled after whole uploads (key_fill).
__device__ inline void put_key(uint32_t* __restrict__ key, int64_t i, float4 a, float4 d, bool cell) {
  if (cell)
    *reinterpret_cast<uint2*>(key + 2 * i) = make_uint2(__float_as_uint(d.z), __float_as_uint(d.w));
  else
    *reinterpret_cast<uint3*>(key + 3 * i) = make_uint3(__float_as_uint(a.x), __float_as_uint(a.y),
                                                        __float_as_uint(a.z));
}

__global__ __launch_bounds__(kBlock) void k_key_fill(const float4* __restrict__ m_a, const float4* __restrict__ m_d,
                                                     int64_t n, int cell, uint32_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  put_key(key, i, m_a[i], cell ? m_d[i] : make_float4(0.f, 0.f, 0.f, 0.f), cell != 0);
}

__global__ __launch_bounds__(kBlock) void k_place_markers_master(const float4* __restrict__ local, int64_t nm,
                                                                 int64_t n_soil, const Body* __restrict__ bodies,
                                                                 Grid g, float4* __restrict__ m_a,
                                                                 float4* __restrict__ m_d,
                                                                 uint32_t* __restrict__ key) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= nm) return;
  float4 l = local[k];
  const Body& b = bodies[__float_as_uint(l.w)];
  double x[3];
  body_point(b, l.x, l.y, l.z, x);
  float4 a = m_a[n_soil + k], d = m_d[n_soil + k];
  store_pos(x, g, a, d);
  m_a[n_soil + k] = a;
  if (g.cell) m_d[n_soil + k] = d;
  if (key) put_key(key, n_soil + k, a, d, g.cell != 0);
}

// Sec. 4.2 item 2: Active inside an oriented box (|R^T (x - X)| <= half per
// local axis), Extended-Active inside the box grown by 2h, else Inactive.
// Activity flag of one FP64 position against all active boxes.
__device__ inline uint8_t flag_of(const double xw[3], const Body* __restrict__ bodies, int32_t nb, double ext) {
#pragma clang fp contract(off)
  uint8_t best = 0;
  for (int b = 0; b < nb; ++b) {
    const Body& B = bodies[b];
    if (!B.has_box) continue;
    // world box around the grown oriented box (a superset: decides nothing)
    if (!(xw[0] >= B.alo[0] && xw[0] <= B.ahi[0] && xw[1] >= B.alo[1] && xw[1] <= B.ahi[1] &&
          xw[2] >= B.alo[2] && xw[2] <= B.ahi[2]))
      continue;
    double d[3], l[3];
    for (int a = 0; a < 3; ++a) d[a] = xw[a] - B.X[a];
    for (int a = 0; a < 3; ++a) l[a] = (B.R[a] * d[0] + B.R[3 + a] * d[1]) + B.R[6 + a] * d[2];
    bool in = true, grown = true;
    for (int a = 0; a < 3; ++a) {
      double al = fabs(l[a]);
      if (!(al <= B.half[a])) in = false;
      if (!(al <= B.half[a] + ext)) grown = false;
    }
    if (in) return 2;
    if (grown) best = 1;
  }
  return best;
}

// The body-by-body pre-test and the exact test of one particle (the flag of
// k_activity_count and of the index's queries).
template <bool CELL>
__device__ inline uint8_t act_flag(const uint32_t* __restrict__ key, const float4* __restrict__ m_a,
                                   const float4* __restrict__ m_d, int64_t i, const Body* __restrict__ bodies,
                                   int32_t nb, const Grid& g) {
  bool cand = false;
  if (CELL) {
    const uint2 kv = *reinterpret_cast<const uint2*>(key + 2 * i);
    const int32_t c0 = (int32_t)kv.x, c1 = unpack_y(kv.y), c2 = unpack_z(kv.y);
    for (int b = 0; b < nb; ++b) {
      const Body& B = bodies[b];
      if (!B.has_box) continue;
      cand |= c0 >= B.clo[0] && c0 <= B.chi[0] && c1 >= B.clo[1] && c1 <= B.chi[1] && c2 >= B.clo[2] &&
              c2 <= B.chi[2];
    }
  } else {
    const uint3 kv = *reinterpret_cast<const uint3*>(key + 3 * i);
    const float x = __uint_as_float(kv.x), y = __uint_as_float(kv.y), z = __uint_as_float(kv.z);
    for (int b = 0; b < nb; ++b) {
      const Body& B = bodies[b];
      if (!B.has_box) continue;
      cand |= x >= B.flo[0] && x <= B.fhi[0] && y >= B.flo[1] && y <= B.fhi[1] && z >= B.flo[2] && z <= B.fhi[2];
    }
  }
  if (!cand) return 0;
  const float4 a = m_a[i];
  const float4 d = CELL ? m_d[i] : a;
  double xw[3];
  abs_pos(a, d, g, xw);
  return flag_of(xw, bodies, nb, g.ext);
}

// Sec. 4.2 item 2 over all N particles, fused with the first pass of the
// order-preserving compaction: block b covers the tile of kFlagsTile particles
// from b kFlagsTile (the tile of k_flags_write), thread t takes the particles
// b kFlagsTile + k kBlock + t, k = 0..15 (each load of a wave reads 64
// consecutive records), and the block's count of flagged particles goes to
// bcnt[b]. A pre-test without FP64 (the world box's FP32 bounds rounded
// outwards for FP32 coordinates, its range of cell indices for cell-offset
// positions) rejects almost every particle of a long terrain; the others take
// the exact FP64 test of flag_of, so every flag is flag_of's. All sixteen
// loads are issued before the first test, the test against the union of the
// bodies' bounds runs on the loaded values, and the few particles inside that
// union take the rest in a loop that reloads them, so that no wait for a
// store or a later load sits between the loads of a thread.
template <bool CELL>
__device__ inline bool in_union(float4 p, const ActUnion& un) {
  if (CELL) {
    const uint32_t w = __float_as_uint(p.w);
    const int32_t c0 = (int32_t)__float_as_uint(p.z), c1 = unpack_y(w), c2 = unpack_z(w);
    return c0 >= un.clo[0] && c0 <= un.chi[0] && c1 >= un.clo[1] && c1 <= un.chi[1] && c2 >= un.clo[2] &&
           c2 <= un.chi[2];
  }
  return p.x >= un.flo[0] && p.x <= un.fhi[0] && p.y >= un.flo[1] && p.y <= un.fhi[1] && p.z >= un.flo[2] &&
         p.z <= un.fhi[2];
}

template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_activity_count(const float4* __restrict__ m_a,
                                                           const float4* __restrict__ m_d,
                                                           const uint32_t* __restrict__ key, int64_t n,
                                                           const Body* __restrict__ bodies, int32_t nb, ActUnion un,
                                                           Grid g, uint8_t* __restrict__ flags,
                                                           uint32_t* __restrict__ bcnt) {
  const int64_t base = (int64_t)blockIdx.x * kFlagsTile + threadIdx.x;
  float4 p[kFlagsPer];   // the compact copy: x, y, z (FP32 coordinates) or the cells in p.zw
#pragma unroll
  for (int q = 0; q < kFlagsPer; ++q) {
    const int64_t i = base + (int64_t)q * kBlock;
    p[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) {
      if (CELL) {
        const uint2 kv = *reinterpret_cast<const uint2*>(key + 2 * i);
        p[q].z = __uint_as_float(kv.x);
        p[q].w = __uint_as_float(kv.y);
      } else {
        const uint3 kv = *reinterpret_cast<const uint3*>(key + 3 * i);
        p[q] = make_float4(__uint_as_float(kv.x), __uint_as_float(kv.y), __uint_as_float(kv.z), 0.f);
      }
    }
  }
  // almost every particle of a long terrain is outside the union: flag 0.
  // All tests come before the first store (a byte store may alias the
  // kernel's arguments for the compiler, which would then reload them and
  // wait for the store first).
  uint32_t near = 0;
#pragma unroll
  for (int q = 0; q < kFlagsPer; ++q)
    if (base + (int64_t)q * kBlock < n && in_union<CELL>(p[q], un)) near |= 1u << q;
#pragma unroll
  for (int q = 0; q < kFlagsPer; ++q) {
    const int64_t i = base + (int64_t)q * kBlock;
    if (i < n && !((near >> q) & 1u)) flags[i] = 0;
  }
  uint32_t cnt = 0;
#pragma unroll 1
  while (near) {
    const int q = __builtin_ctz(near);
    near &= near - 1u;
    const int64_t i = base + (int64_t)q * kBlock;
    const uint8_t f = act_flag<CELL>(key, m_a, m_d, i, bodies, nb, g);
    flags[i] = f;
    cnt += f != 0 ? 1u : 0u;
  }
  uint32_t tot;
  block_excl_scan(cnt, tot);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = tot;
}

// ---------------------------------------------- activity by coarse cells ---
// The same flags without reading all N particles: an index of the master
// store by coarse cell (kCoarse list cells per axis) lists each particle under
// the cell it was in when the index was built. Only integrated particles and
// the markers of moving bodies change position, and each of those is put on a
// moved list (and marked) the first time; every other particle is still where
// the index says. A rebuild then tests the particles listed under the coarse
// cells that the bodies' pre-test cell ranges touch (skipping marked ones) and
// every particle of the moved list, with the same pre-test and flag_of as
// k_activity_count, and counts the flagged particles per compaction tile.
// Particles it does not test lie outside every body's pre-test range, where
// k_activity_count's flag is 0 too; the previous rebuild's flags are cleared
// first, so the flags, and the compaction of them, are the same.
constexpr int kCoarse = 8;

// Coarse cell of master particle i (its list cell clamped to the domain's grid).
template <bool CELL>
__device__ inline uint32_t coarse_of(const float4* __restrict__ m_a, const float4* __restrict__ m_d, int64_t i,
                                     const Grid& g, int32_t cx, int32_t cy) {
  int32_t c[3];
  if (CELL) {
    const float4 d = m_d[i];
    const uint32_t w = __float_as_uint(d.w);
    c[0] = clamp_cell((int32_t)__float_as_uint(d.z), g.gdim[0]);
    c[1] = clamp_cell(unpack_y(w), g.gdim[1]);
    c[2] = clamp_cell(unpack_z(w), g.gdim[2]);
  } else {
    const float4 a = m_a[i];
    c[0] = cell_coord((double)a.x, g.lo[0], g.inv, g.gdim[0]);
    c[1] = cell_coord((double)a.y, g.lo[1], g.inv, g.gdim[1]);
    c[2] = cell_coord((double)a.z, g.lo[2], g.inv, g.gdim[2]);
  }
  return ((uint32_t)(c[2] / kCoarse) * (uint32_t)cy + (uint32_t)(c[1] / kCoarse)) * (uint32_t)cx +
         (uint32_t)(c[0] / kCoarse);
}

// One atomic add per distinct address among the wave's active lanes; returns
// each lane's old value plus its place among the lanes sharing its address.
__device__ inline uint32_t wave_atomic_slot(uint32_t* __restrict__ base, uint32_t c) {
  uint64_t todo = __ballot(1);
  uint64_t mine = 0;
  while (todo) {
    const int lead = __builtin_ctzll(todo);
    const uint32_t lc = (uint32_t)__shfl((int)c, lead);
    const uint64_t set = __ballot(c == lc) & todo;
    if (c == lc) mine = set;
    todo &= ~set;
  }
  const int first = __builtin_ctzll(mine);
  uint32_t b = 0;
  if ((int)lane_id() == first) b = atomicAdd(&base[c], (uint32_t)__popcll(mine));
  b = (uint32_t)__shfl((int)b, first);
  return b + (uint32_t)__popcll(mine & lanemask_lt());
}

template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_ix_count(const float4* __restrict__ m_a, const float4* __restrict__ m_d,
                                                     int64_t n, Grid g, int32_t cx, int32_t cy,
                                                     uint32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  (void)wave_atomic_slot(cnt, coarse_of<CELL>(m_a, m_d, i, g, cx, cy));
}

template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_ix_place(const float4* __restrict__ m_a, const float4* __restrict__ m_d,
                                                     int64_t n, Grid g, int32_t cx, int32_t cy,
                                                     const uint32_t* __restrict__ start, uint32_t* __restrict__ fill,
                                                     int32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = coarse_of<CELL>(m_a, m_d, i, g, cx, cy);
  ids[start[c] + wave_atomic_slot(fill, c)] = (int32_t)i;
}

// Writes a nonzero flag f of particle i and counts it in its compaction tile
// (one atomic add per tile among the wave's lanes; every lane of the wave
// calls this, with f = 0 for none).
__device__ inline void put_flag(uint8_t f, int64_t i, uint8_t* __restrict__ flags, uint32_t* __restrict__ bcnt) {
  if (f) flags[i] = f;
  const uint32_t t = f ? (uint32_t)(i / kFlagsTile) : 0u;
  uint64_t todo = __ballot(f != 0);
  while (todo) {
    const int lead = __builtin_ctzll(todo);
    const uint32_t lt = (uint32_t)__shfl((int)t, lead);
    const uint64_t set = __ballot(f != 0 && t == lt) & todo;
    if ((int)lane_id() == lead) atomicAdd(&bcnt[lt], (uint32_t)__popcll(set));
    todo &= ~set;
  }
}

// Workgroups kQuerySplit * w .. kQuerySplit * w + kQuerySplit - 1 test the
// particles listed under coarse cell visit[w] (those not marked as moved),
// each a strided share: a coarse cell holds thousands of particles, and the
// tests of one particle are a chain of dependent loads, so the cell's share
// per lane is kept to a few.
constexpr int kQuerySplit = 16;

template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_ix_query(const uint32_t* __restrict__ visit,
                                                     const uint32_t* __restrict__ start,
                                                     const int32_t* __restrict__ ids,
                                                     const uint8_t* __restrict__ moved,
                                                     const uint32_t* __restrict__ key, const float4* __restrict__ m_a,
                                                     const float4* __restrict__ m_d, const Body* __restrict__ bodies,
                                                     int32_t nb, Grid g, uint8_t* __restrict__ flags,
                                                     uint32_t* __restrict__ bcnt) {
  const uint32_t c = visit[blockIdx.x / kQuerySplit];
  const uint32_t b = start[c] + (blockIdx.x % kQuerySplit) * kBlock, e = start[c + 1];
  for (uint32_t k0 = b; k0 < e; k0 += kQuerySplit * kBlock) {   // the same trip count for every lane
    const uint32_t k = k0 + threadIdx.x;
    int32_t i = 0;
    uint8_t f = 0;
    if (k < e) {
      i = ids[k];
      const uint8_t mv = moved[i];                     // loaded beside the key
      f = act_flag<CELL>(key, m_a, m_d, i, bodies, nb, g);
      if (mv) f = 0;
    }
    put_flag(f, i, flags, bcnt);
  }
}

// The same for the first min(*n_dev, cap) particles of an id list.
template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_ix_list(const int32_t* __restrict__ list,
                                                    const uint64_t* __restrict__ n_dev, int64_t cap,
                                                    const uint32_t* __restrict__ key, const float4* __restrict__ m_a,
                                                    const float4* __restrict__ m_d, const Body* __restrict__ bodies,
                                                    int32_t nb, Grid g, uint8_t* __restrict__ flags,
                                                    uint32_t* __restrict__ bcnt) {
  const int64_t n = (int64_t)*n_dev < cap ? (int64_t)*n_dev : cap;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k0 = (int64_t)blockIdx.x * kBlock; k0 < n; k0 += stride) {   // uniform per block
    const int64_t k = k0 + threadIdx.x;
    int32_t i = 0;
    uint8_t f = 0;
    if (k < n) {
      i = list[k];
      f = act_flag<CELL>(key, m_a, m_d, i, bodies, nb, g);
    }
    put_flag(f, i, flags, bcnt);
  }
}

// Clears the flags of the first *n_dev ids of a list (the previous rebuild's
// processed particles).
__global__ __launch_bounds__(kBlock) void k_flags_clear(const int32_t* __restrict__ ids,
                                                        const uint64_t* __restrict__ n_dev, int64_t cap,
                                                        uint8_t* __restrict__ flags) {
  const int64_t n = (int64_t)*n_dev < cap ? (int64_t)*n_dev : cap;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
    flags[ids[k]] = 0;
}

// Puts particles on the moved list the first time: the ids of the active soil
// rows (rows, through slot_id), or the ids id0 .. id0 + n - 1 (rows null).
__global__ __launch_bounds__(kBlock) void k_moved_add(const int32_t* __restrict__ rows,
                                                      const uint64_t* __restrict__ n_dev, int64_t n_cap,
                                                      const int32_t* __restrict__ slot_id, int64_t id0,
                                                      uint8_t* __restrict__ moved, int32_t* __restrict__ list,
                                                      uint64_t* __restrict__ n_moved, int64_t cap) {
  const int64_t n = n_dev ? ((int64_t)*n_dev < n_cap ? (int64_t)*n_dev : n_cap) : n_cap;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
    const int32_t id = rows ? slot_id[rows[k]] : (int32_t)(id0 + k);
    if (moved[id]) continue;
    moved[id] = 1;
    const uint64_t p = atomicAdd((unsigned long long*)n_moved, 1ull);
    if ((int64_t)p < cap) list[p] = id;
  }
}

// Largest squared displacement of a processed particle since the last list
// rebuild (A against the rebuild positions in pos4 / cpos), as the bits of a
// non-negative float folded in with an integer atomic max (exact and
// independent of the order).
template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_max_disp(CPlanes A, const float4* __restrict__ pos4,
                                                     const int4* __restrict__ cpos, int64_t n, float Sf,
                                                     uint32_t* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  float d2 = 0.f;
  if (s < n) {
    const float4 a = A.a[s], p = pos4[s];
    float dx = a.x - p.x, dy = a.y - p.y, dz = a.z - p.z;
    if (CELL) {
      const float4 d = A.d[s];
      const int4 c = cpos[s];
      const uint32_t w = __float_as_uint(d.w);
      dx += (float)((int32_t)__float_as_uint(d.z) - c.x) * Sf;
      dy += (float)(unpack_y(w) - c.y) * Sf;
      dz += (float)(unpack_z(w) - c.z) * Sf;
    }
    d2 = dx * dx + dy * dy + dz * dz;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) d2 = fmaxf(d2, __shfl_xor(d2, o, kWave));
  if (lane_id() == 0) atomicMax(out, __float_as_uint(d2));
}

// Processed-marker range of each body: markers are processed in id order and
// body b owns ids n_soil + [bstart[b], bstart[b + 1]), so its processed
// markers are entries [lower_bound(ids, n_soil + bstart[b]) - kbase, ...).
__global__ void k_body_ranges(const int32_t* __restrict__ ids, int64_t n_proc, int64_t n_soil,
                              const int64_t* __restrict__ bstart, int32_t nb, int64_t kbase,
                              int64_t* __restrict__ out) {
  const int32_t b = (int32_t)((int64_t)blockIdx.x * kBlock + threadIdx.x);
  if (b > nb) return;
  const int64_t target = n_soil + bstart[b];
  int64_t lo = 0, hi = n_proc;
  if (ids) {
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if ((int64_t)ids[mid] < target) lo = mid + 1;
      else hi = mid;
    }
  } else {
    lo = target;
  }
  out[b] = lo - kbase;
}

// ------------------------------------------------------ hashing and sort ---
// Sec. 4.1 step 1: c = z * (Y * X) + y * X + x with cell size 2h. The arrival
// rank of each particle in its cell comes from an atomic counter (counting sort).

// A cell of the domain's grid in the rebuild's window (clamped to it; every
// processed particle's cell lies inside, at least one cell from its edges
// unless the edge is the domain's).
__device__ inline int32_t win_cell(int32_t c, const Grid& g, int k) { return clamp_cell(c - g.org[k], g.dims[k]); }

__global__ __launch_bounds__(kBlock) void k_hash_count(const int32_t* __restrict__ ids, int64_t n,
                                                       const float4* __restrict__ m_a,
                                                       const float4* __restrict__ m_d, Grid g,
                                                       uint32_t* __restrict__ key, uint32_t* __restrict__ rank,
                                                       uint32_t* __restrict__ cnt) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  int64_t id = ids ? ids[k] : k;
  int32_t cx, cy, cz;
  if (g.cell) {   // the stored cell, clamped to the grid
    const float4 d = m_d[id];
    const uint32_t w = __float_as_uint(d.w);
    cx = win_cell(clamp_cell((int32_t)__float_as_uint(d.z), g.gdim[0]), g, 0);
    cy = win_cell(clamp_cell(unpack_y(w), g.gdim[1]), g, 1);
    cz = win_cell(clamp_cell(unpack_z(w), g.gdim[2]), g, 2);
  } else {
    const float4 p = m_a[id];
    cx = win_cell(cell_coord((double)p.x, g.lo[0], g.inv, g.gdim[0]), g, 0);
    cy = win_cell(cell_coord((double)p.y, g.lo[1], g.inv, g.gdim[1]), g, 1);
    cz = win_cell(cell_coord((double)p.z, g.lo[2], g.inv, g.gdim[2]), g, 2);
  }
  uint32_t c = ((uint32_t)cz * (uint32_t)g.dims[1] + (uint32_t)cy) * (uint32_t)g.dims[0] + (uint32_t)cx;
  key[k] = c;
  // the lanes of the wave that share a cell take one atomic between them: the
  // lowest lane of each set adds the set's size, and each lane's rank is the
  // returned base plus its place in the set (the order inside a cell is the
  // gather's x order, whatever the ranks)
  uint64_t todo = __ballot(1);
  uint64_t mine = 0;
  while (todo) {                                        // once per distinct cell
    const int lead = __builtin_ctzll(todo);
    const uint32_t lc = (uint32_t)__shfl((int)c, lead);
    const uint64_t set = __ballot(c == lc) & todo;
    if (c == lc) mine = set;
    todo &= ~set;
  }
  const int lane = (int)lane_id();
  const int first = __builtin_ctzll(mine);
  uint32_t base = 0;
  if (lane == first) base = atomicAdd(&cnt[c], (uint32_t)__popcll(mine));
  base = (uint32_t)__shfl((int)base, first);
  rank[k] = base + (uint32_t)__popcll(mine & lanemask_lt());
}

// Order-preserving maps of FP32 / FP64 values onto unsigned integers (total
// orders, NaNs included), and back.
__device__ inline uint32_t f32_order_key(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline unsigned long long f64_order_key(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ inline double f64_from_order_key(unsigned long long k) {
  return __longlong_as_double((long long)((k >> 63) ? (k & ~(1ull << 63)) : ~k));
}

// Arrival position of particle k in its cell, with an order key of its x
// coordinate beside it: the FP32 coordinate for absolute positions (K =
// uint32_t); for cell-offset positions the stored x cell and then the FP32
// offset inside it (K = uint64_t), which orders by x also where stored cells
// outside the grid share an edge cell of the hash.
template <typename K>
__device__ inline K x_order_key(float4 a, float4 d);
template <>
__device__ inline uint32_t x_order_key<uint32_t>(float4 a, float4) {
  return f32_order_key(a.x);
}
template <>
__device__ inline uint64_t x_order_key<uint64_t>(float4 a, float4 d) {
  const uint32_t cx = __float_as_uint(d.z) ^ 0x80000000u;   // signed cell -> unsigned order
  return ((uint64_t)cx << 32) | f32_order_key(a.x);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_place(const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
                                                  const uint32_t* __restrict__ cs, int64_t n,
                                                  const int32_t* __restrict__ ids, const float4* __restrict__ m_a,
                                                  const float4* __restrict__ m_d, uint32_t* __restrict__ tmp,
                                                  K* __restrict__ tmpx) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int64_t id = ids ? ids[k] : k;
  const uint32_t at = cs[key[k]] + rank[k];
  tmp[at] = (uint32_t)k;
  tmpx[at] = x_order_key<K>(m_a[id], sizeof(K) == 8 ? m_d[id] : make_float4(0.f, 0.f, 0.f, 0.f));
}

// Sec. 4.1 step 2 (sort by cell): the order inside a cell, which the hash sort
// leaves open, is made deterministic and spatial: by x, ties by particle id
// (a cell holds ~10-20 particles). A (y, z) row of cells is then ordered by x
// from end to end, so a block's neighbour ranges can be cut to the x interval
// its rows reach. The master state is gathered into the cell-sorted working
// planes.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_gather_sorted(
    const uint32_t* __restrict__ tmp, const K* __restrict__ tmpx, const uint32_t* __restrict__ key,
    const int32_t* __restrict__ ids, const uint32_t* __restrict__ cs, int64_t n, int64_t n_soil,
    const uint8_t* __restrict__ flags, const float4* __restrict__ m_a, const float4* __restrict__ m_b,
    const float4* __restrict__ m_c, const float4* __restrict__ m_d, Planes A, Planes B, float4* __restrict__ pos4,
    int4* __restrict__ cpos, int cell, int32_t* __restrict__ slot_id, int32_t* __restrict__ slot_k,
    uint32_t* __restrict__ skey) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  uint32_t k = tmp[p];
  const K xk = tmpx[p];
  int64_t id = ids ? ids[k] : (int64_t)k;
  // the record's loads go out before the rank is counted
  float4 a = m_a[id], b = m_b[id], cc = m_c[id], d = m_d[id];
  uint32_t c = key[k];
  uint32_t lo = cs[c], hi = cs[c + 1];
  uint32_t r = 0;
#pragma unroll 4
  for (uint32_t q = lo; q < hi; ++q) {   // ids ascend with k
    const K xq = tmpx[q];
    r += (xq < xk || (xq == xk && tmp[q] < k)) ? 1u : 0u;
  }
  uint32_t f = lo + r;
  slot_id[f] = (int32_t)id;
  slot_k[f] = (int32_t)k;
  skey[f] = c;
  uint32_t aux = __float_as_uint(b.w) & ~3u;
  uint32_t kind = (id < n_soil) ? ((flags == nullptr || flags[id] == 2) ? kSoilActive : kSoilExtended) : kMarker;
  b.w = __uint_as_float(aux | kind);
  A.a[f] = a; A.b[f] = b; A.c[f] = cc; A.d[f] = d;
  // stage 1 writes an active soil row's midpoint record before anything reads
  // it; extended soil rows and markers keep y_n there
  if (kind != kSoilActive) {
    B.a[f] = a; B.b[f] = b; B.c[f] = cc; B.d[f] = d;
  }
  pos4[f] = make_float4(a.x, a.y, a.z, b.w);
  if (cell) {
    const uint32_t w = __float_as_uint(d.w);
    cpos[f] = make_int4((int32_t)__float_as_uint(d.z), unpack_y(w), unpack_z(w), 0);
  }
}

// ------------------------------------------------------- neighbour lists ---
// Algorithm 1: for each row particle, the 27 cells around its own; the three
// cells x-1..x+1 of a (y, z) row are consecutive in the sorted order, so they
// are scanned as one range [cellStart[c(x-1)], cellStart[c(x+1) + 1]). The group
// tests kGroup consecutive candidates at a time; membership |x_i - x_j| < 2h is
// decided in FP64 on the FP32 positions. Entries come out in slot order. With
// soil_only (marker rows) only soil candidates are kept: the BCE sums of
// Sec. 2.5.1 run over soil particles, so marker-marker pairs are never used.
__device__ inline double dist2_cell(float4 pi, int4 ci, float4 pj, int4 cj, double S) {
#pragma clang fp contract(off)
  const double dx = (double)(ci.x - cj.x) * S + ((double)pi.x - (double)pj.x);
  const double dy = (double)(ci.y - cj.y) * S + ((double)pi.y - (double)pj.y);
  const double dz = (double)(ci.z - cj.z) * S + ((double)pi.z - (double)pj.z);
  return (dx * dx + dy * dy) + dz * dz;
}

// The group's scan of the 27 cells around cell c for the neighbours of a row
// at (pi, ci). Every candidate is first tested in FP32 against the widened
// radius band [R2lo, R2hi]; only a distance inside the band takes the exact
// FP64 test, so every decision is that of the FP64 test. The FP32 distance
// is within a few FP32 ulps of the exact one: |dx| rounds once (FP32 mode),
// or to within (|dc| + 2) ulps of S (cell mode, dc the cell difference of
// the stored positions), and squaring and summing add a few ulps of the result;
// the band's half-width 2^-14 R2 exceeds these bounds by far.
// Candidates straight from the planes. run(k, b, e) gives the loader of the
// (dz, dy) run k = 3 (dz + 1) + dy + 1 and may narrow [b, e) to a part known
// to hold every neighbour (here the whole run stays).
template <bool CELL>
struct ScanLoad {
  const float4* pos4;
  const int4* cpos;
  __device__ void operator()(uint32_t j, float4& p, int4& cj) const {
    p = at(pos4, j);
    if (CELL) cj = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(cpos) + (j << 4));
  }
  __device__ ScanLoad run(int, uint32_t&, uint32_t&) const { return *this; }
};

// Half-width of the x window of run (dy, dz) for a row at y, z (FP64, from
// the grid's low corner) in global cell row cy, cz. Every candidate of cell
// row cy + dy lies beyond the boundary between the two rows: at least
// e_y = (cy + 1) S - y (dy = 1) or y - cy S (dy = -1) from the row in y, and
// likewise in z, also where cells are clamped to the grid (a clamped row's
// gap only grows). A neighbour within R therefore has
// (x_i - x_j)^2 < R^2 - e_y^2 - e_z^2; the bound is taken with R widened to
// R' = R (1 + 2^-20) and the gaps shrunk by S 2^-20, far above the FP64
// rounding of the cell assignment and of the membership test. A run no
// neighbour can reach gets a negative half-width.
__device__ inline double run_half_width(int dy, int dz, double y, double z, int32_t cy, int32_t cz, double S) {
#pragma clang fp contract(off)
  const double m = S * 0x1p-20;
  const double Rm = S * (1.0 + 0x1p-20);
  double ey = dy > 0 ? (double)(cy + 1) * S - y : dy < 0 ? y - (double)cy * S : 0.0;
  double ez = dz > 0 ? (double)(cz + 1) * S - z : dz < 0 ? z - (double)cz * S : 0.0;
  ey = ey - m > 0.0 ? ey - m : 0.0;
  ez = ez - m > 0.0 ? ez - m : 0.0;
  const double w2 = (Rm * Rm - ey * ey) - ez * ez;
  return w2 > 0.0 ? sqrt(w2) : -1.0;
}

// x of slot j in FP64: absolute, or cell index times cell size plus offset.
template <bool CELL>
__device__ inline double slot_x(const float4* __restrict__ pos4, const int4* __restrict__ cpos, uint32_t j,
                                double S) {
  if constexpr (CELL) return (double)cpos[j].x * S + (double)pos4[j].x;
  else return (double)pos4[j].x;
}

// Candidates straight from the planes, each run cut to the row's x window
// [x_i - W_k, x_i + W_k] (W_k = run_half_width): a run's slots ascend in x
// (cells in x order, each cell's slots in x order), so two binary searches
// over its positions give the part that can hold neighbours. Lane l of the
// row's group narrows runs l and (lane 0) 8 before the scan; run(k) hands the
// group run k's bounds from the lane that narrowed it.
template <bool CELL>
struct ScanNarrowLoad {
  ScanLoad<CELL> ld;
  uint32_t b0, e0, b1, e1;         // this lane's runs (gl and gl + 8)
  __device__ void prepare(bool live, float4 pi, int4 ci, uint32_t c, const uint32_t* __restrict__ cs,
                          const Grid& g) {
    const uint32_t X = (uint32_t)g.dims[0], Y = (uint32_t)g.dims[1], Z = (uint32_t)g.dims[2];
    const int gl = group_lane();
    b0 = e0 = b1 = e1 = 0;
    if (!live) return;
    const int cx = (int)(c % X), cy = (int)((c / X) % Y), cz = (int)(c / (X * Y));
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < (int)X - 1 ? cx + 1 : (int)X - 1;
    const double xi = CELL ? (double)ci.x * g.S + (double)pi.x : (double)pi.x;
    const double yi = CELL ? (double)ci.y * g.S + (double)pi.y : (double)pi.y - g.lo[1];
    const double zi = CELL ? (double)ci.z * g.S + (double)pi.z : (double)pi.z - g.lo[2];
    for (int u = 0; u < 2; ++u) {
      const int k = gl + kGroup * u;
      if (k > 8) break;
      const int z = cz + k / 3 - 1, y = cy + k % 3 - 1;
      uint32_t b = 0, e = 0;
      const double w = run_half_width(k % 3 - 1, k / 3 - 1, yi, zi, cy + g.org[1], cz + g.org[2], g.S);
      if (z >= 0 && z < (int)Z && y >= 0 && y < (int)Y && w >= 0.0) {
        const double wlo = xi - w, whi = xi + w;
        const uint32_t row = ((uint32_t)z * Y + (uint32_t)y) * X;
        b = cs[row + x0];
        e = cs[row + x1 + 1];
        uint32_t a = b, z1 = e;     // first slot at or above wlo
        while (a < z1) {
          const uint32_t m = a + (z1 - a) / 2;
          if (slot_x<CELL>(ld.pos4, ld.cpos, m, g.S) < wlo) a = m + 1;
          else z1 = m;
        }
        b = a;
        uint32_t a2 = b, z2 = e;    // first slot above whi
        while (a2 < z2) {
          const uint32_t m = a2 + (z2 - a2) / 2;
          if (slot_x<CELL>(ld.pos4, ld.cpos, m, g.S) <= whi) a2 = m + 1;
          else z2 = m;
        }
        e = a2;
      }
      if (u == 0) { b0 = b; e0 = e; }
      else { b1 = b; e1 = e; }
    }
  }
  __device__ ScanLoad<CELL> run(int k, uint32_t& b, uint32_t& e) const {
    const int src = (lane_id() & ~(kGroup - 1)) + (k & (kGroup - 1));
    b = (uint32_t)__shfl((int)(k < kGroup ? b0 : b1), src);
    e = (uint32_t)__shfl((int)(k < kGroup ? e0 : e1), src);
    return ld;
  }
};

template <bool FILL, bool CELL, bool SOIL_ONLY, class Load, class Emit>
__device__ inline uint32_t group_scan(bool live, float4 pi, int4 ci, uint32_t c, const Load& load,
                                      const uint32_t* __restrict__ cs, const Grid& g, const Emit& emit,
                                      uint32_t limit) {
  const int X = g.dims[0], Y = g.dims[1], Z = g.dims[2];
  const int gl = group_lane();
  int cx = 0, cy = 0, cz = 0;
  if (live) {
    cx = (int)(c % (uint32_t)X);
    const uint32_t t = c / (uint32_t)X;
    cy = (int)(t % (uint32_t)Y);
    cz = (int)(t / (uint32_t)Y);
  }
  const int x0 = cx > 0 ? cx - 1 : 0;
  const int x1 = cx < X - 1 ? cx + 1 : X - 1;
  const float lo2 = g.R2lo, hi2 = g.R2hi, Sf = g.Sf;
  uint32_t count = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    for (int dy = -1; dy <= 1; ++dy) {
      const int k = 3 * (dz + 1) + dy + 1;
      const int z = cz + dz, y = cy + dy;
      uint32_t b = 0, e = 0;
      if (live && z >= 0 && z < Z && y >= 0 && y < Y) {
        const uint32_t row = ((uint32_t)z * (uint32_t)Y + (uint32_t)y) * (uint32_t)X;
        b = cs[row + x0];
        e = cs[row + x1 + 1];
      }
      const auto run = load.run(k, b, e);
      const auto put = emit.run(k);
      for (uint32_t j0 = b; j0 < e; j0 += kGroup) {
        const uint32_t j = j0 + gl;
        bool hit = false;
        if (j < e) {
          float4 pj;
          int4 cj = make_int4(0, 0, 0, 0);
          run(j, pj, cj);
          if (!SOIL_ONLY || (__float_as_uint(pj.w) & 3u) != kMarker) {
            float sx = pi.x - pj.x, sy = pi.y - pj.y, sz = pi.z - pj.z;
            if (CELL) {
              sx += (float)(ci.x - cj.x) * Sf;
              sy += (float)(ci.y - cj.y) * Sf;
              sz += (float)(ci.z - cj.z) * Sf;
            }
            const float d2 = sx * sx + sy * sy + sz * sz;
            hit = d2 < lo2;
            if (!hit && d2 <= hi2)
              hit = (CELL ? dist2_cell(pi, ci, pj, cj, g.S) : dist2_fp64(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z)) < g.R2;
          }
        }
        const uint32_t m = group_bits(__ballot(hit));
        if (FILL && hit) {
          const uint32_t at_ = count + __popc(m & ((1u << gl) - 1u));
          if (at_ < limit) put(at_, j);
        }
        count += __popc(m);
      }
    }
  }
  return count;
}

// The row scan with the position form and the candidate filter as template
// arguments (uniform over a launch).
template <bool FILL, class Emit>
__device__ inline uint32_t group_scan_any(bool live, float4 pi, int4 ci, uint32_t c, const float4* __restrict__ pos4,
                                          const int4* __restrict__ cpos, const uint32_t* __restrict__ cs,
                                          const Grid& g, bool soil_only, const Emit& emit, uint32_t limit) {
  if (g.cell) {
    const ScanLoad<true> ld{pos4, cpos};
    return soil_only ? group_scan<FILL, true, true>(live, pi, ci, c, ld, cs, g, emit, limit)
                     : group_scan<FILL, true, false>(live, pi, ci, c, ld, cs, g, emit, limit);
  }
  const ScanLoad<false> ld{pos4, cpos};
  return soil_only ? group_scan<FILL, false, true>(live, pi, ci, c, ld, cs, g, emit, limit)
                   : group_scan<FILL, false, false>(live, pi, ci, c, ld, cs, g, emit, limit);
}

// The same with every run cut to the row's x window (ScanNarrowLoad).
template <class Emit>
__device__ inline uint32_t group_scan_narrow(bool live, float4 pi, int4 ci, uint32_t c,
                                             const float4* __restrict__ pos4, const int4* __restrict__ cpos,
                                             const uint32_t* __restrict__ cs, const Grid& g, bool soil_only,
                                             const Emit& emit, uint32_t limit) {
  if (g.cell) {
    ScanNarrowLoad<true> ld{{pos4, cpos}, 0, 0, 0, 0};
    ld.prepare(live, pi, ci, c, cs, g);
    return soil_only ? group_scan<true, true, true>(live, pi, ci, c, ld, cs, g, emit, limit)
                     : group_scan<true, true, false>(live, pi, ci, c, ld, cs, g, emit, limit);
  }
  ScanNarrowLoad<false> ld{{pos4, cpos}, 0, 0, 0, 0};
  ld.prepare(live, pi, ci, c, cs, g);
  return soil_only ? group_scan<true, false, true>(live, pi, ci, c, ld, cs, g, emit, limit)
                   : group_scan<true, false, false>(live, pi, ci, c, ld, cs, g, emit, limit);
}

// Writes entry `at` of a row's list (slot j). run(k) gives the writer of the
// entries found in run k.
struct EmitTo {
  uint32_t* out;
  __device__ void operator()(uint32_t at, uint32_t j) const { out[at] = j; }
  __device__ EmitTo run(int) const { return *this; }
};

// Writes entry `at` as the tile position 16 (j - o_k) of a staged block's cut
// layout (o: the nine o_k, in LDS, read once per run).
struct EmitTilePos {
  uint16_t* out;
  const uint32_t* o;
  struct Run {
    uint16_t* out;
    uint32_t ok;
    __device__ void operator()(uint32_t at, uint32_t j) const { out[at] = (uint16_t)((j - ok) << 4); }
  };
  __device__ Run run(int k) const { return Run{out, o[k]}; }
};

// Count pass: counts every row's neighbours and keeps the first kStash of them
// in a fixed-stride scratch, so that the fill pass is a copy (rows with more
// are scanned again there). The grid covers rows_cap rows; the live row count
// is read on the device and only the blocks that carry live rows are spread
// over the XCDs.
constexpr uint32_t kStash = 80;
static_assert(kStash % kGroup == 0, "whole stash rows per lane");

__global__ __launch_bounds__(kBlock) void k_nbr_count(const int32_t* __restrict__ rows, int64_t rows_cap,
                                                      const uint64_t* __restrict__ n_rows_dev,
                                                      const float4* __restrict__ pos4, const int4* __restrict__ cpos,
                                                      const uint32_t* __restrict__ skey,
                                                      const uint32_t* __restrict__ cs, Grid g, int soil_only,
                                                      uint32_t* __restrict__ cnt, uint32_t* __restrict__ stash) {
  const int64_t nr = (int64_t)*n_rows_dev;
  const int64_t nb_live = (nr * kGroup + kBlock - 1) / kBlock;
  const int64_t r = (xcd_block_n(nb_live) * kBlock + threadIdx.x) / kGroup;
  const bool live = r < nr;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  int4 ci = make_int4(0, 0, 0, 0);
  uint32_t c = 0;
  uint32_t* out = stash;
  if (live) {
    const int32_t s = rows[r];
    pi = pos4[s];
    if (g.cell) ci = cpos[s];
    c = skey[s];
    out = stash + (uint64_t)r * kStash;
  }
  const uint32_t count = group_scan_narrow(live, pi, ci, c, pos4, cpos, cs, g, soil_only != 0, EmitTo{out}, kStash);
  if (r < rows_cap && group_lane() == 0) cnt[r] = live ? count : 0u;
}

__global__ __launch_bounds__(kBlock) void k_nbr_fill(const int32_t* __restrict__ rows, int64_t n_rows,
                                                     const float4* __restrict__ pos4, const int4* __restrict__ cpos,
                                                     const uint32_t* __restrict__ skey,
                                                     const uint32_t* __restrict__ cs, Grid g, int soil_only,
                                                     const uint32_t* __restrict__ cnt,
                                                     const uint32_t* __restrict__ stash,
                                                     const uint64_t* __restrict__ off, uint32_t* __restrict__ nbr) {
  const int64_t r = (xcd_block() * kBlock + threadIdx.x) / kGroup;
  const bool live = r < n_rows;
  const uint32_t count = live ? cnt[r] : 0u;
  // all of the lane's stash words are loaded at once, without waiting for the
  // count (the words past it are read but never stored)
  constexpr int kPer = (int)(kStash / kGroup);
  uint32_t v[kPer];
  if (live) {
    const uint32_t* src = stash + (uint64_t)r * kStash;
#pragma unroll
    for (int q = 0; q < kPer; ++q) v[q] = src[(uint32_t)group_lane() + (uint32_t)(q * kGroup)];
  }
  const bool rescan = count > kStash;                 // uniform within the group
  if (live && !rescan) {
    const uint64_t base = off[r];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const uint32_t k = (uint32_t)group_lane() + (uint32_t)(q * kGroup);
      if (k < count) nbr[base + k] = v[q];
    }
  }
  if (rescan) {
    const int32_t s = rows[r];
    const int4 ci = g.cell ? cpos[s] : make_int4(0, 0, 0, 0);
    group_scan_any<true>(true, pos4[s], ci, skey[s], pos4, cpos, cs, g, soil_only != 0, EmitTo{nbr + off[r]},
                         0xffffffffu);
  }
}

// ------------------------------------------------------------ markers ---
// A marker's lever arm from its body's origin, from the stored position (FP64).
template <bool CELL>
__device__ inline void marker_arm(const Own& me, const Body& Bd, const Phys& P, double rv[3]) {
  if (CELL) {
    rv[0] = from_cell(me.cx, me.x, P.lo[0], P.S) - Bd.X[0];
    rv[1] = from_cell(me.cy, me.y, P.lo[1], P.S) - Bd.X[1];
    rv[2] = from_cell(me.cz, me.z, P.lo[2], P.S) - Bd.X[2];
  } else {
    rv[0] = (double)me.x - Bd.X[0];
    rv[1] = (double)me.y - Bd.X[1];
    rv[2] = (double)me.z - Bd.X[2];
  }
}

// Rigid-body velocity ub = V + W x r and acceleration as = A + Al x r +
// W x (W x r) at lever arm r (FP64, rounded once).
__device__ inline void body_motion(const Body& Bd, const double rv[3], float ub[3], float as[3]) {
  const double wr[3] = {Bd.W[1] * rv[2] - Bd.W[2] * rv[1], Bd.W[2] * rv[0] - Bd.W[0] * rv[2],
                        Bd.W[0] * rv[1] - Bd.W[1] * rv[0]};
  const double wwr[3] = {Bd.W[1] * wr[2] - Bd.W[2] * wr[1], Bd.W[2] * wr[0] - Bd.W[0] * wr[2],
                         Bd.W[0] * wr[1] - Bd.W[1] * wr[0]};
  for (int a = 0; a < 3; ++a) ub[a] = (float)(Bd.V[a] + wr[a]);
  if (Bd.has_acc) {
    const double ar[3] = {Bd.Al[1] * rv[2] - Bd.Al[2] * rv[1], Bd.Al[2] * rv[0] - Bd.Al[0] * rv[2],
                          Bd.Al[0] * rv[1] - Bd.Al[1] * rv[0]};
    for (int a = 0; a < 3; ++a) as[a] = (float)(Bd.A[a] + ar[a] + wwr[a]);
  } else {
    for (int a = 0; a < 3; ++a) as[a] = (float)wwr[a];
  }
}

// Places every processed marker at x = X + R l (both stage states). A marker
// row without soil neighbours (cnt[r] = 0) takes no part in any sum (the
// neighbour relation is symmetric), so the BCE passes skip it: its
// extrapolated values are those of an empty sum, the body velocity at the
// marker and zero stress, written here for both stage states.
template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_place_markers_working(const int32_t* __restrict__ mrows, int64_t n,
                                                                  const uint32_t* __restrict__ cnt,
                                                                  const int32_t* __restrict__ slot_id, int64_t n_soil,
                                                                  const float4* __restrict__ local,
                                                                  const Body* __restrict__ bodies, Grid g, Phys P,
                                                                  Planes A, Planes B, int all) {
  int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  int32_t s = mrows[r];
  float4 l = local[slot_id[s] - n_soil];
  const Body& Bd = bodies[__float_as_uint(l.w)];
  // a body whose pose and velocity are those of the last placement keeps its
  // markers' values (positions, and the body velocity of rows without soil
  // neighbours); after a list rebuild every row is placed once
  if (!all && !Bd.place) return;
  double x[3];
  body_point(Bd, l.x, l.y, l.z, x);
  float4 a = A.a[s], d = A.d[s];
  store_pos(x, g, a, d);
  A.a[s] = a;
  B.a[s] = a;
  const bool far = cnt[r] == 0;
  if (far) {
    double rv[3];
    float ub[3], as[3];
    marker_arm<CELL>(own_pos<CELL>(a, d), Bd, P, rv);
    body_motion(Bd, rv, ub, as);
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    A.b[s] = make_float4(ub[0], ub[1], ub[2], A.b[s].w);
    B.b[s] = make_float4(ub[0], ub[1], ub[2], B.b[s].w);
    A.c[s] = zero;
    B.c[s] = zero;
    d.x = 0.f;
    d.y = 0.f;
  }
  if (CELL || far) {
    A.d[s] = d;
    B.d[s] = d;
  }
}

// One record per marker row with soil neighbours (rebuilt with the lists).
__global__ __launch_bounds__(kBlock) void k_near_rows(const int32_t* __restrict__ mrows,
                                                      const int32_t* __restrict__ near, int64_t n,
                                                      const uint64_t* __restrict__ off, NearRow* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t r = near[i];
  const uint64_t k0 = off[r];
  rows[i] = NearRow{k0, mrows[r], (uint32_t)(off[r + 1] - k0)};
}

// Sec. 2.5.1: Adami velocity u~ = sum u_f W / sum W, no-slip u_s = 2 u_body - u~;
// stress s_s = [sum s_f W - ((g - a_s) . sum rho_f (x_s - x_f) W) I] / sum W.
// With `contrib`, the marker acceleration from the momentum equation over the
// soil neighbours (no body force) and the marker's force and torque on its
// body, at entry cidx[s] - cbase (the marker's rank among the processed
// markers in id order). A marker row (~30 soil neighbours) takes a group of
// kBG lanes; sixteen lanes, one two-entry step per row instead of two, made
// both passes ~25 % slower (the per-row FP64 tail then costs twice as many
// waves).
constexpr int kBG = kGroup;

template <bool FORCE, bool CELL>
__global__ __launch_bounds__(kBlock) void k_bce(Planes S, const NearRow* __restrict__ rows, int64_t n,
                                                const uint32_t* __restrict__ nbr,
                                                const Body* __restrict__ bodies, const int32_t* __restrict__ cidx,
                                                int64_t cbase, Phys P, double* __restrict__ contrib) {
  const int64_t i = (xcd_block() * kBlock + threadIdx.x) / kBG;
  const int gl = group_lane<kBG>();
  const bool live = i < n;
  // a group past the last row reads the last row, walks no entries and
  // stores nothing
  const NearRow nr = rows[live ? i : n - 1];
  const int32_t s = nr.s;
  const float4 ma = S.a[s], mb = S.b[s];
  const float4 md = CELL ? S.d[s] : ma;     // the cells (cell-offset positions only)
  const int body = (int)(__float_as_uint(mb.w) >> 2);
  const uint64_t k0 = nr.k0, k1 = live ? nr.k0 + nr.n : nr.k0;
  const Own me = own_pos<CELL>(ma, md);
  // body velocity and acceleration at the marker (FP64 lever arm), before the
  // walk, so that the body record's loads and the FP64 work overlap it
  double rv[3];
  float ub[3], as[3];
  {
    const Body& Bd = bodies[body];
    marker_arm<CELL>(me, Bd, P, rv);
    body_motion(Bd, rv, ub, as);
  }
  float sw = 0.f, su0 = 0.f, su1 = 0.f, su2 = 0.f;
  float ss0 = 0.f, ss1 = 0.f, ss2 = 0.f, ss3 = 0.f, ss4 = 0.f, ss5 = 0.f;
  float sr0 = 0.f, sr1 = 0.f, sr2 = 0.f;
  walk_row<kBG>(CPlanes(S), k0, k1, nbr, [&](const Nbr& o, uint32_t) {
    float dx, dy, dz;
    pair_sep<CELL>(me, o, P.Sf, dx, dy, dz);
    const float q = fsqrt(dx * dx + dy * dy + dz * dz) * P.inv_h;
    const float w = sph_w(q, P);
    sw += w;
    su0 += o.b.x * w; su1 += o.b.y * w; su2 += o.b.z * w;
    ss0 += o.c.x * w; ss1 += o.c.y * w; ss2 += o.c.z * w;
    ss3 += o.c.w * w; ss4 += o.d.x * w; ss5 += o.d.y * w;
    const float rw = o.a.w * w;
    sr0 += rw * dx; sr1 += rw * dy; sr2 += rw * dz;
  });
  sw = group_sum<kBG>(sw);
  su0 = group_sum<kBG>(su0); su1 = group_sum<kBG>(su1); su2 = group_sum<kBG>(su2);
  ss0 = group_sum<kBG>(ss0); ss1 = group_sum<kBG>(ss1); ss2 = group_sum<kBG>(ss2);
  ss3 = group_sum<kBG>(ss3); ss4 = group_sum<kBG>(ss4); ss5 = group_sum<kBG>(ss5);
  sr0 = group_sum<kBG>(sr0); sr1 = group_sum<kBG>(sr1); sr2 = group_sum<kBG>(sr2);
  float us[3] = {0.f, 0.f, 0.f}, sg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (live) {
    if (sw > 0.f) {
      const float iw = 1.0f / sw;
      const float gd = ((P.gx - as[0]) * sr0 + (P.gy - as[1]) * sr1) + (P.gz - as[2]) * sr2;
      us[0] = 2.f * ub[0] - su0 * iw;
      us[1] = 2.f * ub[1] - su1 * iw;
      us[2] = 2.f * ub[2] - su2 * iw;
      sg[0] = (ss0 - gd) * iw; sg[1] = (ss1 - gd) * iw; sg[2] = (ss2 - gd) * iw;
      sg[3] = ss3 * iw; sg[4] = ss4 * iw; sg[5] = ss5 * iw;
    } else {
      us[0] = ub[0]; us[1] = ub[1]; us[2] = ub[2];
    }
    if (gl == 1) S.b[s] = make_float4(us[0], us[1], us[2], mb.w);
    if (gl == 2) S.c[s] = make_float4(sg[0], sg[1], sg[2], sg[3]);
    if (gl == 3) {
      float4 d = S.d[s];
      d.x = sg[4];
      d.y = sg[5];
      S.d[s] = d;
    }
  }
  if (FORCE) {
    // Momentum equation at the marker (F3) with artificial viscosity, soil
    // neighbours only: a_s = (1/rho_s) sum V_f (s_s + s_f) gradW + Pi.
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, v0 = 0.f, v1 = 0.f, v2 = 0.f;
    const float rhos = live ? ma.w : 1.0f;
    walk_row<kBG>(CPlanes(S), k0, k1, nbr, [&](const Nbr& o, uint32_t) {
      float dx, dy, dz;
      pair_sep<CELL>(me, o, P.Sf, dx, dy, dz);
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float q = fsqrt(r2) * P.inv_h;
      const float F = sph_f(q, P);
      const float VF = P.m * __builtin_amdgcn_rcpf(o.a.w) * F;
      const float wx = VF * dx, wy = VF * dy, wz = VF * dz;
      const float sxx = sg[0] + o.c.x, syy = sg[1] + o.c.y, szz = sg[2] + o.c.z;
      const float sxy = sg[3] + o.c.w, sxz = sg[4] + o.d.x, syz = sg[5] + o.d.y;
      a0 += sxx * wx + sxy * wy + sxz * wz;
      a1 += sxy * wx + syy * wy + syz * wz;
      a2 += sxz * wx + syz * wy + szz * wz;
      const float vr = (us[0] - o.b.x) * dx + (us[1] - o.b.y) * dy + (us[2] - o.b.z) * dz;
      const bool av = P.av_mode == 1 || (P.av_mode == 2 && vr < 0.f);
      const float cf = av ? P.av_coef * vr * F * __builtin_amdgcn_rcpf(0.5f * (rhos + o.a.w) * (r2 + P.xi2)) : 0.f;
      v0 += cf * dx; v1 += cf * dy; v2 += cf * dz;
    });
    a0 = group_sum<kBG>(a0); a1 = group_sum<kBG>(a1); a2 = group_sum<kBG>(a2);
    v0 = group_sum<kBG>(v0); v1 = group_sum<kBG>(v1); v2 = group_sum<kBG>(v2);
    if (live && gl == 0) {
      // force and torque of this marker on its body, by marker id
      const float ir = 1.0f / rhos;
      const double f0 = (double)P.m * (double)(a0 * ir + v0);
      const double f1 = (double)P.m * (double)(a1 * ir + v1);
      const double f2 = (double)P.m * (double)(a2 * ir + v2);
      double* out = contrib + ((int64_t)cidx[s] - cbase) * 6;
      out[0] = f0;
      out[1] = f1;
      out[2] = f2;
      out[3] = rv[1] * f2 - rv[2] * f1;
      out[4] = rv[2] * f0 - rv[0] * f2;
      out[5] = rv[0] * f1 - rv[1] * f0;
    }
  }
}

// Deterministic segmented sums of 6 doubles per entry (the markers' force
// and torque per body; also parameter sums by group): each segment is cut into
// chunks of at most kRedChunk entries; a block sums one chunk in a fixed order
// (strided per thread, then a tree), then each segment sums its chunks' partials
// in chunk order.
constexpr int64_t kRedChunk = 4 * kBlock;

__global__ __launch_bounds__(kBlock) void k_chunk_reduce(const double* __restrict__ in,
                                                         const int64_t* __restrict__ lo,
                                                         const int64_t* __restrict__ hi,
                                                         double* __restrict__ partial) {
  __shared__ double red[6][kBlock];
  const int64_t c = blockIdx.x;
  const int t = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t e = hi[c];
  for (int64_t k = lo[c] + t; k < e; k += kBlock)
    for (int a = 0; a < 6; ++a) acc[a] += in[k * 6 + a];
  for (int a = 0; a < 6; ++a) red[a][t] = acc[a];
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (t < o)
      for (int a = 0; a < 6; ++a) red[a][t] += red[a][t + o];
    __syncthreads();
  }
  if (t < 6) partial[c * 6 + t] = red[t][0];
}

// One block per segment: thread t sums chunks first + t, first + t + kBlock,
// ... in order, then a tree over the threads.
// With seq, the block then adds one to seq[g] behind a system-scope fence, so
// that a host polling seq (host memory mapped for the device, like out) finds
// the segment's sums written once the count moves.
__global__ __launch_bounds__(kBlock) void k_segment_sum(const double* __restrict__ partial,
                                                        const int32_t* __restrict__ first,
                                                        double* __restrict__ out, uint64_t* seq) {
  __shared__ double red[6][kBlock];
  const int32_t g = blockIdx.x;
  const int t = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int32_t c = first[g] + t; c < first[g + 1]; c += kBlock)
    for (int a = 0; a < 6; ++a) acc[a] += partial[(int64_t)c * 6 + a];
  for (int a = 0; a < 6; ++a) red[a][t] = acc[a];
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (t < o)
      for (int a = 0; a < 6; ++a) red[a][t] += red[a][t + o];
    __syncthreads();
  }
  if (t < 6) out[(int64_t)g * 6 + t] = red[t][0];
  if (seq) {
    __threadfence_system();
    __syncthreads();
    if (t == 0) {
      volatile uint64_t* q = seq + g;
      *q = *q + 1u;
      __threadfence_system();
    }
  }
}

// ------------------------------------------------------------- fluid ---
struct Rates {
  float dx, dy, dz;              // position rate = own velocity
  float ax, ay, az;              // acceleration
  float s0, s1, s2, s3, s4, s5;  // stress rate
  float drho;
  float L[9];                    // velocity gradient, row-major (for the adjoint's tape)
};

// Sec. 2.2: L = sum_j V_j (u_j - u_i) (x) gradW (F2); drho/dt = -rho tr L;
// a = (1/rho_i) sum_j V_j (s_i + s_j) . gradW + g + Pi_a (F3, artificial viscosity
// with the sign that repels approaching pairs); ds/dt = Om s - s Om + 2G D +
// (bulk K - 2G/3) tr D I with D, Om the symmetric and skew parts of L.
// The group's G lanes take the row's neighbours k = lane, lane + G, ...;
// walk(pair) calls pair(record) for each of the lane's neighbours, with the
// neighbour's volume V_j = m / rho_j in place of its density (a.w). One
// reciprocal square root gives q and 1 / q. The own stress's share of F3 is
// s_i . sum_j V_j gradW, taken once per row. The viscosity term of a pair is
// a multiple of r_ij, like V_j gradW = w, so it enters the stress sum as an
// isotropic part: rho_i Pi_ij added to the diagonal of s_j, with
// Pi_ij = 2 av (v_ij . r_ij) / ((rho_i V_j + m)(r_ij^2 + xi^2)) (the mean
// density of the pair is (rho_i V_j + m) / (2 V_j)). Every product-sum is an
// explicit FMA and nothing else is contracted, so each way of walking the
// neighbours (tile or L1) gives the same bits by construction.
template <bool CELL, int G, class Walk>
__device__ inline Rates fluid_rhs(float4 ma, float4 mb, float4 mc, float4 md, Walk&& walk, const Phys& P) {
#pragma clang fp contract(off)
  const Own me = own_pos<CELL>(ma, md);
  const float rhoi = ma.w;
  const float ux = mb.x, uy = mb.y, uz = mb.z;
  const float s0 = mc.x, s1 = mc.y, s2 = mc.z, s3 = mc.w, s4 = md.x, s5 = md.y;
  float L00 = 0.f, L01 = 0.f, L02 = 0.f, L10 = 0.f, L11 = 0.f, L12 = 0.f, L20 = 0.f, L21 = 0.f, L22 = 0.f;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;   // sum_j V_j grad_i W_ij (sigma_i's share of F3, applied once per row)
  const float avr = (2.0f * P.av_coef) * rhoi;
  // kernel gradient factor F(q) with its constants folded: cubic inner piece
  // kf (2.25 q - 3), outer piece -0.75 kf (2 - q)^2 / q = -0.75 kf h t^2 / r
  const float ci1 = 2.25f * P.kf, ci0 = -3.0f * P.kf, co = -0.75f * P.kf * P.h;
  auto pair = [&](const Nbr& o) {
#pragma clang fp contract(off)
    float dx, dy, dz;
    pair_sep<CELL>(me, o, P.Sf, dx, dy, dz);
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float rs = __builtin_amdgcn_rsqf(fmaxf(r2, 1.0e-30f));   // 1 / r (finite for the self pair)
    const float q = (r2 * rs) * P.inv_h;
    float F;
    if (P.kern == 1) {
      F = wendland_f(q, P.kf);
    } else {
      const float t = fmaxf(2.0f - q, 0.0f);
      const float outer = ((t * t) * rs) * co;
      const float inner = fmaf(q, ci1, ci0);
      F = q < 1.0f ? inner : outer;
    }
    const float V = o.a.w;
    const float VF = V * F;                                       // V_j * (gradW / r_ij)
    const float wx = VF * dx, wy = VF * dy, wz = VF * dz;       // V_j grad_i W_ij
    const float dux = o.b.x - ux, duy = o.b.y - uy, duz = o.b.z - uz;
    L00 = fmaf(dux, wx, L00); L01 = fmaf(dux, wy, L01); L02 = fmaf(dux, wz, L02);
    L10 = fmaf(duy, wx, L10); L11 = fmaf(duy, wy, L11); L12 = fmaf(duy, wz, L12);
    L20 = fmaf(duz, wx, L20); L21 = fmaf(duz, wy, L21); L22 = fmaf(duz, wz, L22);
    g0 += wx; g1 += wy; g2 += wz;
    const float vr = -fmaf(duz, dz, fmaf(duy, dy, dux * dx));   // v_ij . r_ij
    const bool av = P.av_mode == 1 || (P.av_mode == 2 && vr < 0.f);
    const float pi = av ? (vr * avr) * __builtin_amdgcn_rcpf(fmaf(rhoi, V, P.m) * (r2 + P.xi2)) : 0.f;
    a0 = fmaf(o.c.x + pi, wx, a0); a0 = fmaf(o.c.w, wy, a0); a0 = fmaf(o.d.x, wz, a0);
    a1 = fmaf(o.c.w, wx, a1); a1 = fmaf(o.c.y + pi, wy, a1); a1 = fmaf(o.d.y, wz, a1);
    a2 = fmaf(o.d.x, wx, a2); a2 = fmaf(o.d.y, wy, a2); a2 = fmaf(o.c.z + pi, wz, a2);
  };
  walk(pair);
  L00 = group_sum<G>(L00); L01 = group_sum<G>(L01); L02 = group_sum<G>(L02);
  L10 = group_sum<G>(L10); L11 = group_sum<G>(L11); L12 = group_sum<G>(L12);
  L20 = group_sum<G>(L20); L21 = group_sum<G>(L21); L22 = group_sum<G>(L22);
  a0 = group_sum<G>(a0); a1 = group_sum<G>(a1); a2 = group_sum<G>(a2);
  g0 = group_sum<G>(g0); g1 = group_sum<G>(g1); g2 = group_sum<G>(g2);
  a0 = fmaf(s4, g2, fmaf(s3, g1, fmaf(s0, g0, a0)));
  a1 = fmaf(s5, g2, fmaf(s1, g1, fmaf(s3, g0, a1)));
  a2 = fmaf(s2, g2, fmaf(s5, g1, fmaf(s4, g0, a2)));
  Rates R;
  const float ir = 1.0f / rhoi;
  R.dx = ux; R.dy = uy; R.dz = uz;
  R.ax = fmaf(a0, ir, P.gx);
  R.ay = fmaf(a1, ir, P.gy);
  R.az = fmaf(a2, ir, P.gz);
  const float trD = (L00 + L11) + L22;
  R.drho = -rhoi * trD;
  // spin components Om_xy, Om_xz, Om_yz and strain rate D
  const float wxy = 0.5f * (L01 - L10), wxz = 0.5f * (L02 - L20), wyz = 0.5f * (L12 - L21);
  const float Dxy = 0.5f * (L01 + L10), Dxz = 0.5f * (L02 + L20), Dyz = 0.5f * (L12 + L21);
  // M = Om s; Om s - s Om = M + M^T
  const float Mxx = fmaf(wxz, s4, wxy * s3);
  const float Myy = fmaf(wyz, s5, -wxy * s3);
  const float Mzz = fmaf(-wyz, s5, -wxz * s4);
  const float Mxy = fmaf(wxz, s5, wxy * s1), Myx = fmaf(wyz, s4, -wxy * s0);
  const float Mxz = fmaf(wxz, s2, wxy * s5), Mzx = fmaf(-wyz, s3, -wxz * s0);
  const float Myz = fmaf(wyz, s2, -wxy * s4), Mzy = fmaf(-wyz, s1, -wxz * s3);
  const float iso = P.iso * trD;
  R.s0 = fmaf(2.f, Mxx, fmaf(P.two_G, L00, iso));
  R.s1 = fmaf(2.f, Myy, fmaf(P.two_G, L11, iso));
  R.s2 = fmaf(2.f, Mzz, fmaf(P.two_G, L22, iso));
  R.s3 = fmaf(P.two_G, Dxy, Mxy + Myx);
  R.s4 = fmaf(P.two_G, Dxz, Mxz + Mzx);
  R.s5 = fmaf(P.two_G, Dyz, Myz + Mzy);
  R.L[0] = L00; R.L[1] = L01; R.L[2] = L02;
  R.L[3] = L10; R.L[4] = L11; R.L[5] = L12;
  R.L[6] = L20; R.L[7] = L21; R.L[8] = L22;
  return R;
}

// Sec. 2.4: four-step return mapping of the trial stress st with taubar^n from
// sn, for material M = (mu_s, mu_2, cohesion, p_cri).
__device__ inline void return_map(float st[6], const float sn[6], const Phys& P, float4 M) {
  const float mu_s = M.x, mu_2 = M.y, cohesion = M.z;
  float ps, tbs, pn, tbn;
  p_taubar(st, ps, tbs);
  if (ps < M.w) {
    for (int a = 0; a < 6; ++a) st[a] = 0.f;
    return;
  }
  p_taubar(sn, pn, tbn);
  float gd = (tbs - tbn) * P.inv_Gdt;
  float mu;
  if (!(gd > 0.f)) {
    mu = mu_s;
  } else if (ps <= 0.f) {
    mu = mu_2;
  } else {
    const float I = gd * P.grain_d * fsqrt(P.rho0 / ps);
    mu = mu_s + (mu_2 - mu_s) / (1.0f + P.I0 / I);
  }
  float tmax = mu * ps + cohesion;
  tmax = tmax > 0.f ? tmax : 0.f;
  if (tbs <= tmax) return;
  const float f = tmax / tbs;
  st[0] = -ps + f * (st[0] + ps);
  st[1] = -ps + f * (st[1] + ps);
  st[2] = -ps + f * (st[2] + ps);
  st[3] *= f;
  st[4] *= f;
  st[5] *= f;
}

// ------------------------------------------------- LDS-staged neighbours ---
// A workgroup serves kRows consecutive soil rows (cell-sorted). When they all
// lie in one (y, z) row of cells, every neighbour of every row lies in one of
// nine contiguous slot ranges: the cells x0 - 1 .. x1 + 1 of the nine (y, z)
// rows around it. The block copies these ranges into LDS once, with coalesced
// loads, and the pair loop reads neighbours from LDS instead of making an L1
// line lookup per plane per pair. Blocks whose rows span two cell rows, or
// whose ranges exceed the tile, read from global memory as before.
//
// The soil list passes (k_nbr_count_soil, k_nbr_fill_soil) give each row
// kGroup lanes, the stage kernels kSG. Eight lanes per row in the stages: four
// lanes on 64-row blocks share the once-per-row work (staging, group sums,
// update, return mapping) among 16 rows per wave and issue ~22 % fewer VALU
// instructions, but a 64-row tile leaves three workgroups per CU (80 % of the
// blocks fit 1024 records) instead of four, and the stages then run 9 %
// slower; on 32-row blocks (two waves per workgroup) 22 % slower.
constexpr int kRows = 32;
constexpr int kSG = 8;
constexpr int kListBlock = kRows * kGroup;
constexpr int kStageBlock = kRows * kSG;
static_assert(kListBlock <= 1024 && kStageBlock % kWave == 0, "whole waves per block");
static_assert(kSG >= 4, "lanes 0-3 of a group store the four planes of a row");

// FP32 positions: 52-byte records (sigma_xz in b.w, where the aux word sits in
// HBM; sigma_yz apart); cell-offset positions: 64-byte records (plane d
// carries the cells). Tile configurations (chosen per context, see
// crm_autotune): 0 no tile, 1 small (768 or 640 records, 40 KB: four blocks
// per CU), 2 large (1024 or 832 records, 53 KB: three blocks per CU). On the
// wheel bin the 32-row blocks' cut ranges hold 526 records on average; 97 % of
// the blocks fit 787 and 98 % fit 1024 (2 % span two cell rows).
template <bool CELL, uint32_t CAP>
struct StageTile;
template <uint32_t CAP>
struct StageTile<false, CAP> {
  static constexpr uint32_t kCap = CAP;
  float4 a[CAP], b[CAP], c[CAP];
  float s5[CAP];
};
template <uint32_t CAP>
struct StageTile<true, CAP> {
  static constexpr uint32_t kCap = CAP;
  float4 a[CAP], b[CAP], c[CAP], d[CAP];
};

// Records per tile: the small tiles are the largest that leave four
// workgroups per CU (160 KB of LDS, allocated in 512-byte granules: at most
// 40 KB each), the large ones three.
template <bool CELL, int CFG>
constexpr uint32_t tile_cap() {
  return CFG == 0 ? 1u : CFG == 1 ? (CELL ? 640u : 787u) : (CELL ? 832u : 1024u);
}
static_assert(sizeof(StageTile<false, tile_cap<false, 1>()>) <= 40960, "four small tiles per CU");
static_assert(sizeof(StageTile<true, tile_cap<true, 1>()>) <= 40960, "four small tiles per CU");
static_assert(sizeof(StageTile<false, tile_cap<false, 2>()>) <= 54272, "three large tiles per CU");
static_assert(sizeof(StageTile<true, tile_cap<true, 2>()>) <= 54272, "three large tiles per CU");

// Per block of kRows rows, computed once per list rebuild (k_tile_tables):
// words 0-8 first slot of each of the nine ranges (~0: outside the grid),
// 9-17 offset o_k (slot j of range k sits at tile index j - o_k), 18 total
// records, 19: 0 when the block's rows span two rows of cells, 1 when they lie
// in one, 2 once the count pass has staged the block, cut its ranges to the x
// interval its rows reach and kept its entries as tile positions
// (k_nbr_count_soil). Only blocks marked 2 have tile positions, and a stage
// uses its tile for such a block when the total fits the tile. The ranges
// start as whole cells x_first - 1 .. x_last + 1.
constexpr uint32_t kTabStaged = 2;
constexpr int kTabWords = 20;

__global__ __launch_bounds__(kBlock) void k_tile_tables(const int32_t* __restrict__ rows,
                                                        const uint64_t* __restrict__ n_dev,
                                                        const uint32_t* __restrict__ skey,
                                                        const uint32_t* __restrict__ cs, Phys P,
                                                        uint32_t* __restrict__ tabs) {
  const int64_t n = (int64_t)*n_dev;
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t r0 = b * kRows;
  if (r0 >= n) return;
  uint32_t* t = tabs + b * kTabWords;
  const int64_t rl = (r0 + kRows - 1 < n) ? r0 + kRows - 1 : n - 1;
  const uint32_t X = (uint32_t)P.gdim[0], Y = (uint32_t)P.gdim[1], Z = (uint32_t)P.gdim[2];
  const uint32_t c0 = skey[rows[r0]], c1 = skey[rows[rl]];
  const uint32_t x0 = c0 % X, y0 = (c0 / X) % Y, z0 = c0 / (X * Y);
  const uint32_t x1 = c1 % X, y1 = (c1 / X) % Y, z1 = c1 / (X * Y);
  uint32_t total = 0;
  uint32_t ok = (y0 == y1 && z0 == z1) ? 1u : 0u;
  const uint32_t xl = x0 > 0 ? x0 - 1 : 0, xh = x1 + 1 < X ? x1 + 1 : X - 1;
  int k = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy, ++k) {
      const int64_t yy = (int64_t)y0 + dy, zz = (int64_t)z0 + dz;
      if (!ok || yy < 0 || yy >= (int64_t)Y || zz < 0 || zz >= (int64_t)Z) {
        t[k] = 0xffffffffu;
        t[9 + k] = 0;
        continue;
      }
      const uint64_t base = ((uint64_t)zz * Y + (uint64_t)yy) * X;
      const uint32_t s0 = cs[base + xl], s1 = cs[base + xh + 1];
      t[k] = s0;
      t[9 + k] = s0 - total;
      total += s1 - s0;
    }
  t[18] = total;
  t[19] = ok;
}

// Slot -> tile index through the nine ranges, as scalars (block-uniform,
// kept in SGPRs). Slot j of range k sits at tile index j - o_k; with d_k the
// step of o from the previous range that exists, o_k is o_0 plus the d_m of
// the ranges m <= k that start at or before j (a range outside the grid
// starts at ~0 and never counts). Written as sums so that no select picks
// between two loaded values. The same holds in tile-index space with the
// ranges' first tile indices b_k, for the copy into the tile.
struct TileLoad {
  uint32_t s1, s2, s3, s4, s5, s6, s7, s8;
  uint32_t b1, b2, b3, b4, b5, b6, b7, b8;
  uint32_t o0, d1, d2, d3, d4, d5, d6, d7, d8;
  __device__ uint32_t offset(uint32_t j, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4, uint32_t a5,
                             uint32_t a6, uint32_t a7, uint32_t a8) const {
    uint32_t o = o0;
    o += j >= a1 ? d1 : 0u;
    o += j >= a2 ? d2 : 0u;
    o += j >= a3 ? d3 : 0u;
    o += j >= a4 ? d4 : 0u;
    o += j >= a5 ? d5 : 0u;
    o += j >= a6 ? d6 : 0u;
    o += j >= a7 ? d7 : 0u;
    o += j >= a8 ? d8 : 0u;
    return o;
  }
  __device__ uint32_t index(uint32_t j) const { return j - offset(j, s1, s2, s3, s4, s5, s6, s7, s8); }
  __device__ uint32_t slot(uint32_t t) const { return t + offset(t, b1, b2, b3, b4, b5, b6, b7, b8); }
};

// The block's index maps from its table (uniform loads).
__device__ inline TileLoad tile_loader(const uint32_t* __restrict__ tb) {
  uint32_t st[9], of[9], d[9], bs[9];
  uint32_t prev = tb[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    st[k] = tb[k];
    of[k] = tb[9 + k];
    const bool none = st[k] == 0xffffffffu;
    d[k] = none ? 0u : of[k] - prev;
    prev = none ? prev : of[k];
    bs[k] = none ? 0xffffffffu : st[k] - of[k];
  }
  TileLoad l;
  l.s1 = st[1]; l.s2 = st[2]; l.s3 = st[3]; l.s4 = st[4]; l.s5 = st[5]; l.s6 = st[6]; l.s7 = st[7]; l.s8 = st[8];
  l.b1 = bs[1]; l.b2 = bs[2]; l.b3 = bs[3]; l.b4 = bs[4]; l.b5 = bs[5]; l.b6 = bs[6]; l.b7 = bs[7]; l.b8 = bs[8];
  l.o0 = of[0];
  l.d1 = d[1]; l.d2 = d[2]; l.d3 = d[3]; l.d4 = d[4]; l.d5 = d[5]; l.d6 = d[6]; l.d7 = d[7]; l.d8 = d[8];
  return l;
}

// The fill pass of the soil rows (the copy of k_nbr_fill, rescans included).
// The count pass keeps a staged block's entries as tile positions, 16 i for
// slot j at tile index i (the record's byte offset in each 16-byte tile
// plane), in 16-bit words: they are copied to `tix`, and the slots are written
// to `nbr` only where a stage may read the block through L1, i.e. when its
// total exceeds skip_cap (the tile of the context's configuration; 0 writes
// every slot). Other blocks' entries are slots, copied to `nbr`. Workgroup b
// serves the kRows rows of tile table b, so the table is uniform.
__global__ __launch_bounds__(kListBlock) void k_nbr_fill_soil(const int32_t* __restrict__ rows, int64_t n_rows,
                                                          const float4* __restrict__ pos4,
                                                          const int4* __restrict__ cpos,
                                                          const uint32_t* __restrict__ skey,
                                                          const uint32_t* __restrict__ cs, Grid g,
                                                          const uint32_t* __restrict__ cnt,
                                                          const uint32_t* __restrict__ stash,
                                                          const uint64_t* __restrict__ off, uint32_t* __restrict__ nbr,
                                                          const uint32_t* __restrict__ tabs,
                                                          uint16_t* __restrict__ tix, uint32_t skip_cap) {
  const int64_t blk = xcd_block();
  const int64_t r = (blk * kListBlock + threadIdx.x) / kGroup;
  const bool live = r < n_rows;
  const uint32_t* tb = tabs + blk * kTabWords;
  const bool tiled = tb[19] == kTabStaged;
  const bool slots = !tiled || tb[18] > skip_cap;
  const TileLoad ld = tile_loader(tb);
  const uint32_t count = live ? cnt[r] : 0u;
  const bool rescan = count > kStash;                 // uniform within the group
  // all of the lane's stash words are loaded at once, without waiting for the
  // count (the words past it are read but never stored)
  constexpr int kPer = (int)(kStash / kGroup);
  if (tiled) {
    uint32_t v[kPer];
    if (live) {
      const uint16_t* src = reinterpret_cast<const uint16_t*>(stash + (uint64_t)r * kStash);
#pragma unroll
      for (int q = 0; q < kPer; ++q) v[q] = src[(uint32_t)group_lane() + (uint32_t)(q * kGroup)];
    }
    if (live && !rescan) {
      const uint64_t base = off[r];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const uint32_t k = (uint32_t)group_lane() + (uint32_t)(q * kGroup);
        if (k < count) {
          tix[base + k] = (uint16_t)v[q];
          if (slots) nbr[base + k] = ld.slot(v[q] >> 4);
        }
      }
    }
  } else {
    uint32_t v[kPer];
    if (live) {
      const uint32_t* src = stash + (uint64_t)r * kStash;
#pragma unroll
      for (int q = 0; q < kPer; ++q) v[q] = src[(uint32_t)group_lane() + (uint32_t)(q * kGroup)];
    }
    if (live && !rescan) {
      const uint64_t base = off[r];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const uint32_t k = (uint32_t)group_lane() + (uint32_t)(q * kGroup);
        if (k < count) nbr[base + k] = v[q];
      }
    }
  }
  if (rescan) {
    const int32_t s = rows[r];
    const int4 ci = g.cell ? cpos[s] : make_int4(0, 0, 0, 0);
    uint32_t* nb = nbr + off[r];
    uint16_t* tx = tix + off[r];
    struct EmitBoth {
      uint32_t* nb;
      uint16_t* tx;
      const TileLoad* ld;
      bool tiled;
      __device__ void operator()(uint32_t at, uint32_t j) const {
        nb[at] = j;
        if (tiled) tx[at] = (uint16_t)(ld->index(j) << 4);
      }
      __device__ EmitBoth run(int) const { return *this; }
    };
    group_scan_any<true>(true, pos4[s], ci, skey[s], pos4, cpos, cs, g, false, EmitBoth{nb, tx, &ld, tiled},
                         0xffffffffu);
  }
}

// The slots of the entries k_nbr_fill_soil left out (staged blocks whose total
// is at most skip_cap), from their tile positions: for the reverse sweep, the
// exported lists, and stages with a smaller tile or none.
__global__ __launch_bounds__(kListBlock) void k_nbr_slots(int64_t n_rows, const uint64_t* __restrict__ off,
                                                      const uint32_t* __restrict__ tabs,
                                                      const uint16_t* __restrict__ tix, uint32_t* __restrict__ nbr,
                                                      uint32_t skip_cap) {
  const int64_t blk = xcd_block();
  const uint32_t* tb = tabs + blk * kTabWords;
  if (tb[19] != kTabStaged || tb[18] > skip_cap) return;    // uniform over the block
  const int64_t r = (blk * kListBlock + threadIdx.x) / kGroup;
  if (r >= n_rows) return;
  const TileLoad ld = tile_loader(tb);
  const uint64_t k1 = off[r + 1];
  for (uint64_t k = off[r] + (uint64_t)group_lane(); k < k1; k += kGroup) nbr[k] = ld.slot((uint32_t)tix[k] >> 4);
}

// ------------------------------------------- LDS-staged neighbour count ---
// The count pass of the soil rows with the candidates of each block's nine
// ranges staged in LDS (positions, and cells with cell-offset positions): a
// row's run of candidates in cells x - 1 .. x + 1 of one (y, z) row lies
// inside the block's range of that (y, z) row, at tile index slot - o_k. Blocks
// whose rows span two cell rows, or whose ranges exceed scan_cap records,
// read the candidates from the planes. On the wheel bin the whole-cell ranges
// of a 32-row block hold 633 records on average; 99.8 % of the blocks fit 1024.
template <bool CELL>
constexpr uint32_t scan_cap() { return 1024u; }

template <bool CELL>
struct ScanTile;
template <>
struct ScanTile<false> {
  float4 p[scan_cap<false>()];
};
template <>
struct ScanTile<true> {
  float4 p[scan_cap<true>()];
  int4 c[scan_cap<true>()];
};
static_assert(sizeof(ScanTile<true>) <= 49152 && sizeof(ScanTile<false>) <= 32768, "three count blocks per CU");

// Candidates from the block's LDS tile: run k reads slot j at tile index
// j - o_k and is cut to the block's range k [lo_k, hi_k), which holds every
// neighbour of the block's rows. o, lo, hi: the block's run table in LDS.
template <bool CELL>
struct ScanTileLoad {
  const ScanTile<CELL>* T;
  const uint32_t* rt;              // o[9], lo[9], hi[9]
  struct Run {
    const ScanTile<CELL>* T;
    uint32_t o;
    __device__ void operator()(uint32_t j, float4& p, int4& cj) const {
      const uint32_t t = j - o;
      p = T->p[t];
      if constexpr (CELL) cj = T->c[t];
    }
  };
  __device__ Run run(int k, uint32_t& b, uint32_t& e) const {
    const uint32_t lo = rt[9 + k], hi = rt[18 + k];
    b = b > lo ? b : lo;
    e = e < hi ? e : hi;
    return Run{T, rt[k]};
  }
};

// x of tile record t in FP64: absolute, or cell index times cell size plus
// offset.
template <bool CELL>
__device__ inline double tile_x(const ScanTile<CELL>& T, uint32_t t, double S) {
  if constexpr (CELL) return (double)T.c[t].x * S + (double)T.p[t].x;
  else return (double)T.p[t].x;
}

// The staged candidates of one row, each run also cut to the row's own x
// window [x_i - R', x_i + R'] (R' as for the block's cut): only the first
// cell of a run can hold slots below it and only the last cell slots above
// it, each in x order, so two binary searches in LDS give the run's part.
// Lane l of the row's group narrows runs l and (lane 0) 8 before the scan;
// run(k) hands the group run k's bounds from the lane that narrowed it. (The
// per-run windows of ScanNarrowLoad do not pay here: the eight rows of a wave
// lie anywhere in y and z within their cell, so the wave still steps through
// each run as long as its longest row needs, and the searches get longer.)
template <bool CELL>
struct ScanRowLoad {
  const ScanTile<CELL>* T;
  const uint32_t* rt;              // o[9], lo[9], hi[9] (block's cut ranges)
  uint32_t b0, e0, b1, e1;         // this lane's runs (gl and gl + 8)
  using Run = typename ScanTileLoad<CELL>::Run;
  __device__ void prepare(bool live, float4 pi, int4 ci, uint32_t c, const uint32_t* __restrict__ cs,
                          const Grid& g) {
    const uint32_t X = (uint32_t)g.dims[0], Y = (uint32_t)g.dims[1], Z = (uint32_t)g.dims[2];
    const int gl = group_lane();
    b0 = e0 = b1 = e1 = 0;
    if (!live) return;
    const int cx = (int)(c % X), cy = (int)((c / X) % Y), cz = (int)(c / (X * Y));
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < (int)X - 1 ? cx + 1 : (int)X - 1;
    const double xi = CELL ? (double)ci.x * g.S + (double)pi.x : (double)pi.x;
    const double Rm = g.S * (1.0 + 0x1p-20);
    const double wlo = xi - Rm, whi = xi + Rm;
    for (int u = 0; u < 2; ++u) {
      const int k = gl + kGroup * u;
      if (k > 8) break;
      const int z = cz + k / 3 - 1, y = cy + k % 3 - 1;
      uint32_t b = 0, e = 0;
      if (z >= 0 && z < (int)Z && y >= 0 && y < (int)Y) {
        const uint32_t row = ((uint32_t)z * Y + (uint32_t)y) * X;
        b = cs[row + x0];
        e = cs[row + x1 + 1];
        const uint32_t m1 = cs[row + x0 + 1], m2 = cs[row + x1];
        const uint32_t o = rt[k], lo = rt[9 + k], hi = rt[18 + k];
        b = b > lo ? b : lo;
        e = e < hi ? e : hi;
        // first slot of the first cell at or above wlo
        uint32_t a = b, z1 = m1 < e ? m1 : e;
        while (a < z1) {
          const uint32_t m = a + (z1 - a) / 2;
          if (tile_x(*T, m - o, g.S) < wlo) a = m + 1;
          else z1 = m;
        }
        b = a;
        // first slot of the last cell above whi
        uint32_t a2 = m2 > b ? m2 : b, z2 = e;
        while (a2 < z2) {
          const uint32_t m = a2 + (z2 - a2) / 2;
          if (tile_x(*T, m - o, g.S) <= whi) a2 = m + 1;
          else z2 = m;
        }
        e = a2 > b ? a2 : b;
      }
      if (u == 0) { b0 = b; e0 = e; }
      else { b1 = b; e1 = e; }
    }
  }
  __device__ Run run(int k, uint32_t& b, uint32_t& e) const {
    const int src = (lane_id() & ~(kGroup - 1)) + (k & (kGroup - 1));
    b = (uint32_t)__shfl((int)(k < kGroup ? b0 : b1), src);
    e = (uint32_t)__shfl((int)(k < kGroup ? e0 : e1), src);
    return Run{T, rt[k]};
  }
};

// Count pass of the soil rows. A block whose rows lie in one row of cells
// and whose ranges (whole cells x_first - 1 .. x_last + 1 of the nine (y, z)
// rows) fit scan_cap records stages their positions in LDS and cuts each
// range to the slots whose x lies within [x_min - R', x_max + R']: x_min,
// x_max are the extremes of the block's rows and R' is the list radius
// widened by 2^-20, far above the FP64 rounding of the separations; every
// neighbour j of a row i has |x_i - x_j| <= R, so every neighbour of the
// block stays in. Cells hold their slots in x order, so only the first cell
// of a range loses a leading run and only the last cell a trailing one. The
// block then scans its rows' runs cut to the ranges and writes the cut
// ranges back into its table, so that the fill pass and the stage kernels
// copy only those records into their tiles.
template <bool CELL>
__global__ __launch_bounds__(kListBlock) void k_nbr_count_soil(const int32_t* __restrict__ rows, int64_t rows_cap,
                                                           const uint64_t* __restrict__ n_rows_dev,
                                                           const float4* __restrict__ pos4,
                                                           const int4* __restrict__ cpos,
                                                           const uint32_t* __restrict__ skey,
                                                           const uint32_t* __restrict__ cs, Grid g,
                                                           uint32_t* __restrict__ tabs,
                                                           uint32_t* __restrict__ cnt, uint32_t* __restrict__ stash) {
  __shared__ ScanTile<CELL> tile;
  __shared__ uint32_t rt[27];     // run table: o_k of the staged layout, cut bounds lo_k, hi_k
  __shared__ uint32_t ct[36];     // per range: first slot, o_k, leading cut, trailing cut
  __shared__ uint32_t os[9];      // o_k of the cut layout (the stage kernels' tiles)
  __shared__ unsigned long long xext[2];   // order keys of the rows' x extremes
  const int64_t nr = (int64_t)*n_rows_dev;
  const int64_t nb_live = (nr + kRows - 1) / kRows;
  const int64_t blk = xcd_block_n(nb_live);
  const int64_t r = (blk * kListBlock + threadIdx.x) / kGroup;
  const bool live = r < nr;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  int4 ci = make_int4(0, 0, 0, 0);
  uint32_t c = 0;
  uint32_t* out = stash;
  if (live) {
    const int32_t s = rows[r];
    pi = pos4[s];
    if (CELL) ci = cpos[s];
    c = skey[s];
    out = stash + (uint64_t)r * kStash;
  }
  bool staged = false;
  if (blk < nb_live) {                      // uniform over the block
    uint32_t* tb = tabs + blk * kTabWords;
    const uint32_t total = tb[18];
    staged = tb[19] != 0 && total <= scan_cap<CELL>();
    if (staged) {
      const TileLoad ld = tile_loader(tb);
      constexpr int kPer = (int)(scan_cap<CELL>() / kListBlock);
      static_assert(scan_cap<CELL>() % kListBlock == 0, "whole records per thread");
      float4 p[kPer];
      int4 q[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const uint32_t t = threadIdx.x + (uint32_t)(u * kListBlock);
        if (t < total) {
          const uint32_t j = ld.slot(t);
          p[u] = pos4[j];
          if (CELL) q[u] = cpos[j];
        }
      }
      // thread t < 18 takes the first (t < 9) or last cell of range k = t % 9
      const int64_t r0 = blk * kRows;
      const int64_t rl = (r0 + kRows - 1 < nr) ? r0 + kRows - 1 : nr - 1;
      const int k = (int)threadIdx.x % 9;
      uint32_t cb0 = 0, cb1 = 0, st = 0xffffffffu, ok_ = 0;
      if (threadIdx.x < 18) {
        st = tb[k];
        ok_ = tb[9 + k];
        const uint32_t X = (uint32_t)g.dims[0], Y = (uint32_t)g.dims[1];
        const uint32_t c0 = skey[rows[r0]], c1 = skey[rows[rl]];
        const uint32_t x0 = c0 % X, y0 = (c0 / X) % Y, z0 = c0 / (X * Y), x1 = c1 % X;
        const uint32_t xl = x0 > 0 ? x0 - 1 : 0, xh = x1 + 1 < X ? x1 + 1 : X - 1;
        if (st != 0xffffffffu) {
          const uint64_t base = ((uint64_t)(z0 + k / 3 - 1) * Y + (uint64_t)(y0 + k % 3 - 1)) * X;
          const uint32_t cx = threadIdx.x < 9 ? xl : xh;
          cb0 = cs[base + cx];
          cb1 = cs[base + cx + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const uint32_t t = threadIdx.x + (uint32_t)(u * kListBlock);
        if (t < total) {
          tile.p[t] = p[u];
          if constexpr (CELL) tile.c[t] = q[u];
        }
      }
      if (threadIdx.x == 0) {
        xext[0] = ~0ull;
        xext[1] = 0ull;
      }
      __syncthreads();
      if (live && group_lane() == 0) {
        const unsigned long long key = f64_order_key(CELL ? (double)ci.x * g.S + (double)pi.x : (double)pi.x);
        atomicMin(&xext[0], key);
        atomicMax(&xext[1], key);
      }
      __syncthreads();
      if (threadIdx.x < 18) {
        const double Rm = g.S * (1.0 + 0x1p-20);
        const bool lead = threadIdx.x < 9;
        const double lim = lead ? f64_from_order_key(xext[0]) - Rm : f64_from_order_key(xext[1]) + Rm;
        // the cell's slots ascend in x: binary search for the first slot with
        // x >= lim (leading cut) or x > lim (trailing cut)
        uint32_t cut = 0;
        if (st != 0xffffffffu) {
          uint32_t a = cb0, b = cb1;
          while (a < b) {
            const uint32_t m = a + (b - a) / 2;
            const double x = tile_x(tile, m - ok_, g.S);
            if (lead ? x < lim : x <= lim) a = m + 1;
            else b = m;
          }
          cut = lead ? a - cb0 : cb1 - a;
        }
        if (lead) {
          ct[k] = st;
          ct[9 + k] = ok_;
          ct[18 + k] = cut;
        } else {
          ct[27 + k] = cut;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t end = total, nlo[9], nhi[9];
#pragma unroll
        for (int m = 8; m >= 0; --m) {
          const uint32_t sm = ct[m], om = ct[9 + m];
          if (sm == 0xffffffffu) {
            nlo[m] = nhi[m] = 0;
          } else {
            const uint32_t first = sm - om;
            nlo[m] = sm + ct[18 + m];
            nhi[m] = sm + (end - first) - ct[27 + m];
            if (nhi[m] < nlo[m]) nhi[m] = nlo[m];
            end = first;
          }
        }
        uint32_t acc = 0;
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          rt[m] = ct[9 + m];
          rt[9 + m] = nlo[m];
          rt[18 + m] = nhi[m];
          os[m] = 0;
          if (ct[m] == 0xffffffffu) continue;
          tb[m] = nlo[m];
          tb[9 + m] = nlo[m] - acc;
          os[m] = nlo[m] - acc;
          acc += nhi[m] - nlo[m];
        }
        tb[18] = acc;
        tb[19] = kTabStaged;
      }
    }
    __syncthreads();
  }
  uint32_t count;
  if (staged) {
    ScanRowLoad<CELL> tl{&tile, rt, 0, 0, 0, 0};
    tl.prepare(live, pi, ci, c, cs, g);
    // the row's entries as 16-bit tile positions of the cut layout
    count = group_scan<true, CELL, false>(live, pi, ci, c, tl, cs, g,
                                          EmitTilePos{reinterpret_cast<uint16_t*>(out), os}, kStash);
  } else {
    ScanNarrowLoad<CELL> nl{{pos4, cpos}, 0, 0, 0, 0};
    nl.prepare(live, pi, ci, c, cs, g);
    count = group_scan<true, CELL, false>(live, pi, ci, c, nl, cs, g, EmitTo{out}, kStash);
  }
  if (r < rows_cap && group_lane() == 0) cnt[r] = live ? count : 0u;
}

// A neighbour's record from the tile at byte offset o of each plane.
template <bool CELL, uint32_t CAP>
__device__ inline Nbr tile_rec(const StageTile<CELL, CAP>& T, uint32_t o) {
  auto at_ = [&](const float4* p) { return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(p) + o); };
  Nbr n;
  n.a = at_(T.a);
  n.b = at_(T.b);
  n.c = at_(T.c);
  if constexpr (CELL) {
    n.d = at_(T.d);
  } else {
    n.d = make_float4(n.b.w, *reinterpret_cast<const float*>(reinterpret_cast<const char*>(T.s5) + (o >> 2)), 0.f,
                      0.f);
  }
  return n;
}

// The walk of a row through the tile, two entries per lane and step: both
// tile reads are issued before either pair is computed, and the tile positions
// four entries ahead are in flight meanwhile (the loop body holds two steps,
// so that the positions in flight need no register moves). The pairs are still
// taken in entry order. pos(k) is the tile position of entry k (relative to
// the block's first entry); e0..e1 are the row's entries; past the row's end
// the walk reads its last entry again (a valid position).
template <int GW, bool CELL, uint32_t CAP, class Pos, class Fn>
__device__ inline void walk_tile_pos(const StageTile<CELL, CAP>& T, const Pos& pos_of, uint32_t e0, uint32_t e1,
                                     Fn&& f) {
  constexpr uint32_t G = (uint32_t)GW;
  const uint32_t ef = e0 + (uint32_t)group_lane<GW>();
  if (ef >= e1) return;
  const uint32_t el = e1 - 1;
  auto pos = [&](uint32_t e) { return pos_of(e < el ? e : el); };
  uint32_t e = ef;
  uint32_t o0 = pos(e), o1 = pos(e + G), o2 = pos(e + 2 * G), o3 = pos(e + 3 * G);
  for (;;) {
    {
      const bool has1 = e + G < e1;
      const bool more = e + 2 * G < e1;
      const Nbr a = tile_rec(T, o0);
      const Nbr b = tile_rec(T, o1);
      o0 = pos(e + 4 * G);
      o1 = pos(e + 5 * G);
      f(a);
      if (has1) f(b);
      if (!more) break;
      e += 2 * G;
    }
    {
      const bool has1 = e + G < e1;
      const bool more = e + 2 * G < e1;
      const Nbr a = tile_rec(T, o2);
      const Nbr b = tile_rec(T, o3);
      o2 = pos(e + 4 * G);
      o3 = pos(e + 5 * G);
      f(a);
      if (has1) f(b);
      if (!more) break;
      e += 2 * G;
    }
  }
}

// Tile positions read from HBM/L2 (`tix` is the block's first entry); the
// load from there is the walk's longest wait. Positions are below 16 total
// (k_nbr_fill_soil, for blocks that stage); LDS reads past the block's
// allocation would return zero, never fault.
template <int GW, bool CELL, uint32_t CAP, class Fn>
__device__ inline void walk_tile(const StageTile<CELL, CAP>& T, const uint16_t* __restrict__ tix, uint32_t e0,
                                 uint32_t e1, Fn&& f) {
  walk_tile_pos<GW>(T, [&](uint32_t k) {
    return (uint32_t)*reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(tix) + 2u * k);
  }, e0, e1, f);
}

// The soil block a stage kernel's workgroup serves: logical block xcd_block()
// through the launch order when there is one (a value past the last block,
// which a launch order of rows in cell order never holds, is clamped).
__device__ inline int64_t stage_block(const int32_t* __restrict__ bperm, int64_t n) {
  const int64_t b = xcd_block();
  if (!bperm) return b;
  const int64_t last = (n + kRows - 1) / kRows - 1;
  const int64_t p = bperm[b];
  return p >= 0 && p <= last ? p : last;
}

// One record on its way into the tile.
struct Rec {
  float4 a, b, c, d;
};

// Record t of the block's ranges (a thread past the total reads record 0
// again, which it does not store: no default values to set up).
template <bool CELL>
__device__ inline Rec rec_load(CPlanes S, const TileLoad& ld, uint32_t t, uint32_t total) {
  Rec r;
  const uint32_t j = ld.slot(t < total ? t : 0u);
  r.a = S.a[j];
  r.b = S.b[j];
  r.c = S.c[j];
  if constexpr (CELL) {
    r.d = S.d[j];
  } else {                         // sigma_xz, sigma_yz: the tile keeps no more of plane d
    const float2 d2 = *reinterpret_cast<const float2*>(&S.d[j]);
    r.d = make_float4(d2.x, d2.y, 0.f, 0.f);
  }
  return r;
}

// The tile holds the neighbour's volume m / rho in place of its density.
__device__ inline float volume(float m, float rho) { return m * __builtin_amdgcn_rcpf(rho); }

template <bool CELL, uint32_t CAP>
__device__ inline void rec_store(StageTile<CELL, CAP>& T, const Rec& r, uint32_t t, uint32_t total, float m) {
  if (t >= total) return;
  T.a[t] = make_float4(r.a.x, r.a.y, r.a.z, volume(m, r.a.w));
  T.c[t] = r.c;
  if constexpr (CELL) {
    T.b[t] = r.b;
    T.d[t] = r.d;
  } else {
    T.b[t] = make_float4(r.b.x, r.b.y, r.b.z, r.d.x);
    T.s5[t] = r.d.y;
  }
}

// Copies the block's ranges into its tile, each thread's (at most four)
// records loaded together before any is stored. Every thread of the block
// calls it; returns whether the block uses the tile.
template <bool CELL, uint32_t CAP>
__device__ inline bool stage_tile(StageTile<CELL, CAP>& T, CPlanes S, const uint32_t* __restrict__ tb,
                                  const TileLoad& ld, float m) {
  static_assert(CAP <= 4 * kStageBlock, "four records per thread");
  static_assert(CAP <= scan_cap<CELL>(), "a tile holds at most the count pass's staged records");
  const uint32_t total = tb[18];
  const bool ok = tb[19] == kTabStaged && total <= CAP;
  if (ok) {
    // the third and fourth rounds only where the total reaches them (uniform)
    const uint32_t t0 = threadIdx.x;
    const bool has2 = total > 2 * kStageBlock, has3 = total > 3 * kStageBlock;
    const Rec r0 = rec_load<CELL>(S, ld, t0, total);
    const Rec r1 = rec_load<CELL>(S, ld, t0 + kStageBlock, total);
    Rec r2, r3;
    if (has2) r2 = rec_load<CELL>(S, ld, t0 + 2 * kStageBlock, total);
    if (has3) r3 = rec_load<CELL>(S, ld, t0 + 3 * kStageBlock, total);
    rec_store(T, r0, t0, total, m);
    rec_store(T, r1, t0 + kStageBlock, total, m);
    if (has2) rec_store(T, r2, t0 + 2 * kStageBlock, total, m);
    if (has3) rec_store(T, r3, t0 + 3 * kStageBlock, total, m);
  }
  __syncthreads();
  return ok;
}

// Tape of a stage for the reverse sweep: L in planes l0..l2 and, in stage 2,
// the trial stress in planes t0..t1; plane k is written by lane k (mod group).
__device__ inline void tape_write(const StageTape& T, int32_t s, const float L[9], const float* st, int np) {
  for (int k = group_lane<kSG>(); k < np; k += kSG) {
    float4 v;
    float4* dst;
    if (k == 0) { v = make_float4(L[0], L[1], L[2], L[3]); dst = T.l0; }
    else if (k == 1) { v = make_float4(L[4], L[5], L[6], L[7]); dst = T.l1; }
    else if (k == 2) { v = make_float4(L[8], 0.f, 0.f, 0.f); dst = T.l2; }
    else if (k == 3) { v = make_float4(st[0], st[1], st[2], st[3]); dst = T.t0; }
    else { v = make_float4(st[4], st[5], 0.f, 0.f); dst = T.t1; }
    dst[s] = v;
  }
}

// Stage-1 update of row s from its record (ma..md) and rates: B = A + dt/2 f;
// lane gl < 4 of the group stores plane gl.
template <bool CELL, bool TAPE>
__device__ inline void finish_stage1(Planes B, int32_t s, int gl, float4 ma, float4 mb, float4 mc, float4 md,
                                     const Rates& R, const Phys& P, const StageTape& T) {
  const float h = P.half_dt;
  float4 na = ma, nd = md;
  advance_pos<CELL>(na, nd, h, R.dx, R.dy, R.dz, P);
  na.w = ma.w + h * R.drho;
  nd.x = md.x + h * R.s4;
  nd.y = md.y + h * R.s5;
  const float4 nb = make_float4(mb.x + h * R.ax, mb.y + h * R.ay, mb.z + h * R.az, mb.w);
  const float4 nc = make_float4(mc.x + h * R.s0, mc.y + h * R.s1, mc.z + h * R.s2, mc.w + h * R.s3);
  float4* dst = gl == 0 ? B.a : gl == 1 ? B.b : gl == 2 ? B.c : B.d;
  const float4 v = gl == 0 ? na : gl == 1 ? nb : gl == 2 ? nc : nd;
  if (gl < 4) dst[s] = v;
  if (TAPE) tape_write(T, s, R.L, nullptr, 3);
}

// Stage-2 update of row s from its y_n record (ya..yd) and the rates at the
// midpoint: A = A + dt f, then the return mapping; lane gl < 4 stores plane gl.
template <bool CELL, bool TAPE>
__device__ inline void finish_stage2(Planes A, int32_t s, int gl, float4 ya, float4 yb, float4 yc, float4 yd,
                                     const Rates& R, const Phys& P, const StageTape& T) {
  const float h = P.dt;
  float4 na = ya, nd = yd;
  advance_pos<CELL>(na, nd, h, R.dx, R.dy, R.dz, P);
  na.w = ya.w + h * R.drho;
  const float sn[6] = {yc.x, yc.y, yc.z, yc.w, yd.x, yd.y};
  float st[6] = {sn[0] + h * R.s0, sn[1] + h * R.s1, sn[2] + h * R.s2,
                 sn[3] + h * R.s3, sn[4] + h * R.s4, sn[5] + h * R.s5};
  float trial[6] = {st[0], st[1], st[2], st[3], st[4], st[5]};
  return_map(st, sn, P, P.mat[__float_as_uint(yb.w) >> 2]);
  nd.x = st[4];
  nd.y = st[5];
  const float4 nb = make_float4(yb.x + h * R.ax, yb.y + h * R.ay, yb.z + h * R.az, yb.w);
  const float4 nc = make_float4(st[0], st[1], st[2], st[3]);
  float4* dst = gl == 0 ? A.a : gl == 1 ? A.b : gl == 2 ? A.c : A.d;
  const float4 v = gl == 0 ? na : gl == 1 ? nb : gl == 2 ? nc : nd;
  if (gl < 4) dst[s] = v;
  if (TAPE) tape_write(T, s, R.L, trial, 5);
}

// Stage 1 of the explicit midpoint rule (Sec. 2.3): B = A + dt/2 f(A).
// Lanes 0-3 of the group write the four planes of the row's record. With TAPE
// the velocity gradient L is also kept.
template <bool CELL, bool TAPE, int CFG>
__global__ __launch_bounds__(kStageBlock) void k_fluid_stage1(CPlanes A, Planes B, const int32_t* __restrict__ rows,
                                                         int64_t n, const uint64_t* __restrict__ off,
                                                         const uint32_t* __restrict__ nbr, Phys P, StageTape T,
                                                         const uint32_t* __restrict__ tabs,
                                                         const uint16_t* __restrict__ tix) {
  constexpr uint32_t CAP = tile_cap<CELL, CFG>();
  __shared__ StageTile<CELL, CAP> tile;
  const int64_t blk = stage_block(P.bperm, n);
  const int64_t r = (blk * kStageBlock + threadIdx.x) / kSG;
  const int gl = group_lane<kSG>();
  const bool live = r < n;
  // a group past the last row reads the last row (no default values to set
  // up), walks no entries and stores nothing
  const int64_t rr = live ? r : n - 1;
  const int32_t s = rows[rr];
  const float4 ma = A.a[s], mb = A.b[s], mc = A.c[s], md = A.d[s];
  const uint64_t k0 = off[rr];
  const uint64_t k1 = live ? off[rr + 1] : k0;
  const uint32_t* tb = tabs + blk * kTabWords;
  const TileLoad tl = tile_loader(tb);
  const bool staged = CFG != 0 && stage_tile(tile, A, tb, tl, P.m);
  Rates R;
  if (staged) {
    const uint64_t kb = off[blk * kRows];
    const uint32_t e0 = live ? uint32_t(k0 - kb) : 0u, e1 = live ? uint32_t(k1 - kb) : 0u;
    R = fluid_rhs<CELL, kSG>(ma, mb, mc, md, [&](auto&& f) { walk_tile<kSG>(tile, tix + kb, e0, e1, f); }, P);
  } else {
    R = fluid_rhs<CELL, kSG>(ma, mb, mc, md, [&](auto&& f) {
      walk_row_with<kSG>(GlobalLoad{A}, k0, k1, nbr, [&](const Nbr& o, uint32_t) {
        Nbr v = o;
        v.a.w = volume(P.m, o.a.w);
        f(v);
      });
    }, P);
  }
  if (!live) return;
  finish_stage1<CELL, TAPE>(B, s, gl, ma, mb, mc, md, R, P, T);
}

// Stage 2: A = A + dt f(B), then the return mapping on the stress. With TAPE
// the velocity gradient and the trial stress are also kept.
template <bool CELL, bool TAPE, int CFG>
__global__ __launch_bounds__(kStageBlock) void k_fluid_stage2(CPlanes B, Planes A, const int32_t* __restrict__ rows,
                                                         int64_t n, const uint64_t* __restrict__ off,
                                                         const uint32_t* __restrict__ nbr, Phys P, StageTape T,
                                                         const uint32_t* __restrict__ tabs,
                                                         const uint16_t* __restrict__ tix) {
  constexpr uint32_t CAP = tile_cap<CELL, CFG>();
  __shared__ StageTile<CELL, CAP> tile;
  const int64_t blk = stage_block(P.bperm, n);
  const int64_t r = (blk * kStageBlock + threadIdx.x) / kSG;
  const int gl = group_lane<kSG>();
  const bool live = r < n;
  // a group past the last row reads the last row (no default values to set
  // up), walks no entries and stores nothing
  const int64_t rr = live ? r : n - 1;
  const int32_t s = rows[rr];
  const float4 ma = B.a[s], mb = B.b[s], mc = B.c[s], md = B.d[s];
  const float4 ya = A.a[s], yb = A.b[s], yc = A.c[s], yd = A.d[s];
  const uint64_t k0 = off[rr];
  const uint64_t k1 = live ? off[rr + 1] : k0;
  const uint32_t* tb = tabs + blk * kTabWords;
  const TileLoad tl = tile_loader(tb);
  const bool staged = CFG != 0 && stage_tile(tile, B, tb, tl, P.m);
  Rates R;
  if (staged) {
    const uint64_t kb = off[blk * kRows];
    const uint32_t e0 = live ? uint32_t(k0 - kb) : 0u, e1 = live ? uint32_t(k1 - kb) : 0u;
    R = fluid_rhs<CELL, kSG>(ma, mb, mc, md, [&](auto&& f) { walk_tile<kSG>(tile, tix + kb, e0, e1, f); }, P);
  } else {
    R = fluid_rhs<CELL, kSG>(ma, mb, mc, md, [&](auto&& f) {
      walk_row_with<kSG>(GlobalLoad{B}, k0, k1, nbr, [&](const Nbr& o, uint32_t) {
        Nbr v = o;
        v.a.w = volume(P.m, o.a.w);
        f(v);
      });
    }, P);
  }
  if (!live) return;
  // Every lane loads the whole y_n record (before the walk, so that the loads
  // overlap it) and computes the whole y_{n+1} record; one store then writes
  // plane gl from lane gl < 4. The return mapping needs sigma_n from planes c
  // and d, so no lane may read a plane after another lane of the group has
  // overwritten it.
  finish_stage2<CELL, TAPE>(A, s, gl, ya, yb, yc, yd, R, P, T);
}

__global__ __launch_bounds__(kBlock) void k_scatter(CPlanes src, const int32_t* __restrict__ rows, int64_t n,
                                                    const int32_t* __restrict__ slot_id,
                                                    float4* __restrict__ m_a, float4* __restrict__ m_b,
                                                    float4* __restrict__ m_c, float4* __restrict__ m_d,
                                                    uint32_t* __restrict__ key, int cell) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const int32_t id = slot_id[s];
  const float4 a = src.a[s], d = src.d[s];
  m_a[id] = a;
  m_b[id] = src.b[s];
  m_c[id] = src.c[s];
  m_d[id] = d;
  if (key) put_key(key, id, a, d, cell != 0);
}

// Marker rows: the extrapolated velocity and stress only. A marker's position
// (a.xyz, and its cells in d.zw) is the body's placement, never the working
// set's copy, which may carry the pose of an earlier step.
__global__ __launch_bounds__(kBlock) void k_scatter_markers(CPlanes src, const int32_t* __restrict__ rows, int64_t n,
                                                            const int32_t* __restrict__ slot_id,
                                                            float4* __restrict__ m_b, float4* __restrict__ m_c,
                                                            float4* __restrict__ m_d) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const int32_t id = slot_id[s];
  m_b[id] = src.b[s];
  m_c[id] = src.c[s];
  const float4 d = src.d[s];
  float4 md = m_d[id];
  md.x = d.x;
  md.y = d.y;
  m_d[id] = md;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned nblk_groups(int64_t rows) { return nblk(rows * kGroup); }
// Workgroups of the soil passes: one per kRows rows (one per tile table).
inline unsigned soil_blocks(int64_t rows) { return (unsigned)((rows + kRows - 1) / kRows); }

}  // namespace

// ------------------------------------------------------------ launchers ---
size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t scan_u32_to_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s) {
  return scan_impl<uint32_t, uint32_t>(in, out, n, tmp, s);
}

hipError_t scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, hipStream_t s) {
  return scan_impl<uint32_t, uint64_t>(in, out, n, tmp, s);
}

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  k_fill_u32<<<(unsigned)b, kBlock, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t copy2_u64(uint64_t* dst, const uint64_t* a, const uint64_t* b, hipStream_t s) {
  k_copy2<<<1, 64, 0, s>>>(dst, a, b);
  return hipGetLastError();
}

hipError_t copy_f64(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_copy_f64<<<nblk(n), kBlock, 0, s>>>(dst, src, n);
  return hipGetLastError();
}

hipError_t place_markers_master(const float4* local, int64_t k0, int64_t k1, int64_t n_soil, const Body* bodies,
                                Grid g, float4* m_a, float4* m_d, uint32_t* key, hipStream_t s) {
  if (k1 <= k0) return hipSuccess;
  k_place_markers_master<<<nblk(k1 - k0), kBlock, 0, s>>>(local + k0, k1 - k0, n_soil + k0, bodies, g, m_a, m_d,
                                                          key);
  return hipGetLastError();
}

hipError_t max_disp(CPlanes A, const float4* pos4, const int4* cpos, int64_t n, bool cell, float Sf, uint32_t* out,
                    hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (cell) k_max_disp<true><<<nblk(n), kBlock, 0, s>>>(A, pos4, cpos, n, Sf, out);
  else k_max_disp<false><<<nblk(n), kBlock, 0, s>>>(A, pos4, cpos, n, Sf, out);
  return hipGetLastError();
}

hipError_t body_ranges(const int32_t* ids, int64_t n_proc, int64_t n_soil, const int64_t* bstart, int32_t nb,
                       int64_t kbase, int64_t* out, hipStream_t s) {
  k_body_ranges<<<nblk((int64_t)nb + 1), kBlock, 0, s>>>(ids, n_proc, n_soil, bstart, nb, kbase, out);
  return hipGetLastError();
}

size_t compact_tmp_elems(int64_t n) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  return (size_t)(2 * nb + 1) + scan_tmp_elems(nb);
}

int64_t coarse_cells(const Grid& g, int32_t cd[3]) {
  for (int k = 0; k < 3; ++k) cd[k] = (g.gdim[k] + kCoarse - 1) / kCoarse;
  return (int64_t)cd[0] * cd[1] * cd[2];
}

int32_t coarse_size() { return kCoarse; }

int64_t flag_tiles(int64_t n) { return (n + kFlagsTile - 1) / kFlagsTile; }

hipError_t ix_build(const float4* m_a, const float4* m_d, int64_t n, Grid g, uint32_t* start, uint32_t* fill,
                    uint32_t* scan_tmp, int32_t* ids, hipStream_t s) {
  int32_t cd[3];
  const int64_t M = coarse_cells(g, cd);
  hipError_t e = fill_u32(fill, 0u, M, s);
  if (e != hipSuccess) return e;
  if (n > 0 && g.cell) k_ix_count<true><<<nblk(n), kBlock, 0, s>>>(m_a, m_d, n, g, cd[0], cd[1], fill);
  else if (n > 0) k_ix_count<false><<<nblk(n), kBlock, 0, s>>>(m_a, m_d, n, g, cd[0], cd[1], fill);
  e = scan_u32_to_u32(fill, start, M, scan_tmp, s);   // every cell's range, empty ones too
  if (e == hipSuccess) e = fill_u32(fill, 0u, M, s);
  if (e != hipSuccess || n <= 0) return e;
  if (g.cell) k_ix_place<true><<<nblk(n), kBlock, 0, s>>>(m_a, m_d, n, g, cd[0], cd[1], start, fill, ids);
  else k_ix_place<false><<<nblk(n), kBlock, 0, s>>>(m_a, m_d, n, g, cd[0], cd[1], start, fill, ids);
  return hipGetLastError();
}

hipError_t ix_flags(const uint32_t* visit, int64_t n_visit, const uint32_t* start, const int32_t* ids,
                    const uint8_t* moved, const int32_t* mlist, const uint64_t* n_moved, int64_t mcap,
                    const uint32_t* key, const float4* m_a, const float4* m_d, const Body* bodies, int32_t nb, Grid g,
                    uint8_t* flags, uint32_t* bcnt, hipStream_t s) {
  if (n_visit > 0) {
    if (g.cell)
      k_ix_query<true><<<(unsigned)(n_visit * kQuerySplit), kBlock, 0, s>>>(visit, start, ids, moved, key, m_a, m_d, bodies, nb, g,
                                                            flags, bcnt);
    else
      k_ix_query<false><<<(unsigned)(n_visit * kQuerySplit), kBlock, 0, s>>>(visit, start, ids, moved, key, m_a, m_d, bodies, nb, g,
                                                             flags, bcnt);
  }
  const unsigned gl = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nblk(mcap), 1024));
  if (g.cell) k_ix_list<true><<<gl, kBlock, 0, s>>>(mlist, n_moved, mcap, key, m_a, m_d, bodies, nb, g, flags, bcnt);
  else k_ix_list<false><<<gl, kBlock, 0, s>>>(mlist, n_moved, mcap, key, m_a, m_d, bodies, nb, g, flags, bcnt);
  return hipGetLastError();
}

hipError_t flags_clear(const int32_t* ids, const uint64_t* n_dev, int64_t cap, uint8_t* flags, hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  const unsigned gl = (unsigned)std::min<int64_t>(nblk(cap), 1024);
  k_flags_clear<<<gl, kBlock, 0, s>>>(ids, n_dev, cap, flags);
  return hipGetLastError();
}

hipError_t moved_add(const int32_t* rows, const uint64_t* n_dev, int64_t n_cap, const int32_t* slot_id, int64_t id0,
                     uint8_t* moved, int32_t* list, uint64_t* n_moved, int64_t cap, hipStream_t s) {
  if (n_cap <= 0) return hipSuccess;
  const unsigned gl = (unsigned)std::min<int64_t>(nblk(n_cap), 1024);
  k_moved_add<<<gl, kBlock, 0, s>>>(rows, n_dev, n_cap, slot_id, id0, moved, list, n_moved, cap);
  return hipGetLastError();
}

hipError_t activity_count(const float4* m_a, const float4* m_d, const uint32_t* key, int64_t n, const Body* bodies,
                          int32_t nb, const ActUnion& un, Grid g, uint8_t* flags, uint32_t* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = (n + kFlagsTile - 1) / kFlagsTile;
  if (g.cell) k_activity_count<true><<<(unsigned)nt, kBlock, 0, s>>>(m_a, m_d, key, n, bodies, nb, un, g, flags, tmp);
  else k_activity_count<false><<<(unsigned)nt, kBlock, 0, s>>>(m_a, m_d, key, n, bodies, nb, un, g, flags, tmp);
  return hipGetLastError();
}

hipError_t compact_counted(const uint8_t* flags, int64_t n, int32_t* out_ids, uint64_t* count_dst, uint32_t* tmp,
                           hipStream_t s) {
  if (n <= 0) {
    k_set_one<uint64_t><<<1, 64, 0, s>>>(count_dst, 0ull);
    return hipGetLastError();
  }
  const int64_t nchunks = (n + kFlagsPer - 1) / kFlagsPer;
  const int64_t nb = (n + kFlagsTile - 1) / kFlagsTile;
  const uint32_t* bcnt = tmp;
  uint32_t* boff = tmp + nb;
  uint32_t* stmp = boff + nb + 1;
  const uint4* f16 = reinterpret_cast<const uint4*>(flags);
  hipError_t e = scan_impl<uint32_t, uint32_t>(bcnt, boff, nb, stmp, s);
  if (e != hipSuccess) return e;
  k_flags_write<<<(unsigned)nb, kBlock, 0, s>>>(f16, nchunks, boff, out_ids);
  k_store_count<<<1, 64, 0, s>>>(count_dst, boff + nb);
  return hipGetLastError();
}

int64_t flags_padded(int64_t n) { return (n + kFlagsPer - 1) / kFlagsPer * kFlagsPer; }

hipError_t compact_kind(const float4* pos4, int64_t n, uint32_t kind, int32_t* rows, uint64_t* count_dst,
                        uint32_t* tmp, hipStream_t s) {
  return compact_impl(PredKind{pos4, kind}, n, rows, count_dst, tmp, s);
}

hipError_t compact_nonzero(const uint32_t* cnt, int64_t n, int32_t* rows, uint64_t* count_dst, uint32_t* tmp,
                           hipStream_t s) {
  return compact_impl(PredNonzero{cnt}, n, rows, count_dst, tmp, s);
}

hipError_t hash_count(const int32_t* ids, int64_t n, const float4* m_a, const float4* m_d, Grid g, uint32_t* key,
                      uint32_t* rank, uint32_t* cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_hash_count<<<nblk(n), kBlock, 0, s>>>(ids, n, m_a, m_d, g, key, rank, cnt);
  return hipGetLastError();
}

hipError_t place_sorted(const uint32_t* key, const uint32_t* rank, const uint32_t* cs, int64_t n, const int32_t* ids,
                        const float4* m_a, const float4* m_d, uint32_t* tmp, uint64_t* tmpx, bool cell, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (cell)
    k_place<uint64_t><<<nblk(n), kBlock, 0, s>>>(key, rank, cs, n, ids, m_a, m_d, tmp, tmpx);
  else
    k_place<uint32_t><<<nblk(n), kBlock, 0, s>>>(key, rank, cs, n, ids, m_a, m_d, tmp,
                                                 reinterpret_cast<uint32_t*>(tmpx));
  return hipGetLastError();
}

hipError_t gather_sorted(const uint32_t* tmp, const uint64_t* tmpx, const uint32_t* key, const int32_t* ids,
                         const uint32_t* cs, int64_t n, int64_t n_soil, const uint8_t* flags, const float4* m_a,
                         const float4* m_b, const float4* m_c, const float4* m_d, Planes A, Planes B,
                         float4* pos4, int4* cpos, int32_t* slot_id, int32_t* slot_k, uint32_t* skey, bool cell,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (cell)
    k_gather_sorted<uint64_t><<<nblk(n), kBlock, 0, s>>>(tmp, tmpx, key, ids, cs, n, n_soil, flags, m_a, m_b, m_c, m_d,
                                                         A, B, pos4, cpos, 1, slot_id, slot_k, skey);
  else
    k_gather_sorted<uint32_t><<<nblk(n), kBlock, 0, s>>>(tmp, reinterpret_cast<const uint32_t*>(tmpx), key, ids, cs,
                                                         n, n_soil, flags, m_a, m_b, m_c, m_d, A, B, pos4, cpos, 0,
                                                         slot_id, slot_k, skey);
  return hipGetLastError();
}

size_t stash_elems(int64_t rows_cap) { return (size_t)rows_cap * kStash; }

hipError_t nbr_count(const int32_t* rows, int64_t rows_cap, const uint64_t* n_rows_dev, const float4* pos4,
                     const int4* cpos, const uint32_t* skey, const uint32_t* cs, Grid g, bool soil_only,
                     uint32_t* cnt, uint32_t* stash, hipStream_t s) {
  if (rows_cap <= 0) return hipSuccess;
  k_nbr_count<<<nblk_groups(rows_cap), kBlock, 0, s>>>(rows, rows_cap, n_rows_dev, pos4, cpos, skey, cs, g,
                                                       soil_only ? 1 : 0, cnt, stash);
  return hipGetLastError();
}

hipError_t nbr_count_soil(const int32_t* rows, int64_t rows_cap, const uint64_t* n_rows_dev, const float4* pos4,
                          const int4* cpos, const uint32_t* skey, const uint32_t* cs, Grid g, uint32_t* tabs,
                          uint32_t* cnt, uint32_t* stash, hipStream_t s) {
  if (rows_cap <= 0) return hipSuccess;
  if (g.cell)
    k_nbr_count_soil<true><<<soil_blocks(rows_cap), kListBlock, 0, s>>>(rows, rows_cap, n_rows_dev, pos4, cpos, skey, cs, g,
                                                                    tabs, cnt, stash);
  else
    k_nbr_count_soil<false><<<soil_blocks(rows_cap), kListBlock, 0, s>>>(rows, rows_cap, n_rows_dev, pos4, cpos, skey, cs,
                                                                     g, tabs, cnt, stash);
  return hipGetLastError();
}

hipError_t nbr_fill(const int32_t* rows, int64_t n_rows, const float4* pos4, const int4* cpos, const uint32_t* skey,
                    const uint32_t* cs, Grid g, bool soil_only, const uint32_t* cnt, const uint32_t* stash,
                    const uint64_t* off, uint32_t* nbr, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  k_nbr_fill<<<nblk_groups(n_rows), kBlock, 0, s>>>(rows, n_rows, pos4, cpos, skey, cs, g, soil_only ? 1 : 0, cnt,
                                                    stash, off, nbr);
  return hipGetLastError();
}

hipError_t place_markers_working(const int32_t* mrows, int64_t n, const uint32_t* cnt, const int32_t* slot_id,
                                 int64_t n_soil, const float4* local, const Body* bodies, Grid g, Phys P, Planes A,
                                 Planes B, bool all, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (g.cell)
    k_place_markers_working<true><<<nblk(n), kBlock, 0, s>>>(mrows, n, cnt, slot_id, n_soil, local, bodies, g, P, A, B,
                                                             all ? 1 : 0);
  else
    k_place_markers_working<false><<<nblk(n), kBlock, 0, s>>>(mrows, n, cnt, slot_id, n_soil, local, bodies, g, P, A,
                                                              B, all ? 1 : 0);
  return hipGetLastError();
}

hipError_t near_rows(const int32_t* mrows, const int32_t* near, int64_t n, const uint64_t* off, NearRow* rows,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_near_rows<<<nblk(n), kBlock, 0, s>>>(mrows, near, n, off, rows);
  return hipGetLastError();
}

hipError_t bce(Planes S, const NearRow* rows, int64_t n, const uint32_t* nbr, const Body* bodies,
               const int32_t* cidx, int64_t cbase, Phys P, double* contrib, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned gsz = nblk(n * kBG);
  if (P.cell) {
    if (contrib)
      k_bce<true, true><<<gsz, kBlock, 0, s>>>(S, rows, n, nbr, bodies, cidx, cbase, P, contrib);
    else
      k_bce<false, true><<<gsz, kBlock, 0, s>>>(S, rows, n, nbr, bodies, cidx, cbase, P, nullptr);
  } else {
    if (contrib)
      k_bce<true, false><<<gsz, kBlock, 0, s>>>(S, rows, n, nbr, bodies, cidx, cbase, P, contrib);
    else
      k_bce<false, false><<<gsz, kBlock, 0, s>>>(S, rows, n, nbr, bodies, cidx, cbase, P, nullptr);
  }
  return hipGetLastError();
}

int64_t reduce_chunk() { return kRedChunk; }


hipError_t segment_reduce(const double* in, const SegPlan& plan, double* out, hipStream_t s, uint64_t* seq) {
  if (plan.nseg <= 0) return hipSuccess;
  if (plan.nchunk > 0)
    k_chunk_reduce<<<(unsigned)plan.nchunk, kBlock, 0, s>>>(in, plan.lo, plan.hi, plan.partial);
  k_segment_sum<<<(unsigned)plan.nseg, kBlock, 0, s>>>(plan.partial, plan.first, out, seq);
  return hipGetLastError();
}

// The body table from the kernel's arguments (up to kBodyPack bodies): the
// upload of a co-simulation step without a copy engine transfer or a staging
// buffer to guard.
__global__ void k_put_bodies(BodyPack p, int32_t nb, Body* __restrict__ dst) {
  const int nw = nb * (int)(sizeof(Body) / sizeof(uint32_t));
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&p.b[0]);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int k = threadIdx.x; k < nw; k += blockDim.x) d[k] = src[k];
}

// ------------------------------------ launch order of the soil blocks ---
// In cell order the blocks that read one record (those of the nine rows of
// cells around it) lie up to a plane of rows apart, farther than an XCD's L2
// holds on wide grids, and the record is fetched from HBM up to three times.
// Ordered by chunks of kOrderW cells along x (then row of cells, then x), the
// plane within a chunk is kOrderW cells wide. Blocks are in cell order, so
// the blocks of one (chunk, row) group are consecutive.
constexpr int kOrderW = 16;

__device__ inline uint32_t block_group(const int32_t* __restrict__ rows, const uint32_t* __restrict__ skey,
                                       int64_t b, uint32_t X, uint32_t R) {
  const uint32_t c = skey[rows[b * kRows]];
  return (c % X) / (uint32_t)kOrderW * R + c / X;
}

__global__ __launch_bounds__(kBlock) void k_block_groups(const int32_t* __restrict__ rows,
                                                         const uint32_t* __restrict__ skey, int64_t nb, uint32_t X,
                                                         uint32_t R, uint32_t* __restrict__ cnt,
                                                         uint32_t* __restrict__ first) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  const uint32_t e = block_group(rows, skey, b, X, R);
  atomicAdd(&cnt[e], 1u);
  if (b == 0 || block_group(rows, skey, b - 1, X, R) != e) first[e] = (uint32_t)b;
}

__global__ __launch_bounds__(kBlock) void k_block_perm(const int32_t* __restrict__ rows,
                                                       const uint32_t* __restrict__ skey, int64_t nb, uint32_t X,
                                                       uint32_t R, const uint32_t* __restrict__ base,
                                                       const uint32_t* __restrict__ first,
                                                       const uint32_t* __restrict__ cnt, int32_t* __restrict__ perm) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  const uint32_t e = block_group(rows, skey, b, X, R);
  const uint32_t k = (uint32_t)b - first[e];
  if (k < cnt[e]) perm[base[e] + k] = (int32_t)b;   // always, for rows in cell order
}

int32_t order_width() { return kOrderW; }

int64_t soil_block_count(int64_t rows) { return (rows + kRows - 1) / kRows; }

int64_t block_order_size(const Grid& g) {
  return (int64_t)((g.dims[0] + kOrderW - 1) / kOrderW) * g.dims[1] * g.dims[2];
}

hipError_t block_order(const int32_t* rows, const uint32_t* skey, int64_t n_rows, Grid g, uint32_t* cnt,
                       uint32_t* first, uint32_t* base, uint32_t* scan_tmp, int32_t* perm, hipStream_t s) {
  const int64_t nb = (n_rows + kRows - 1) / kRows;
  if (nb <= 0) return hipSuccess;
  const int64_t M = block_order_size(g);
  const uint32_t X = (uint32_t)g.dims[0], R = (uint32_t)g.dims[1] * (uint32_t)g.dims[2];
  hipError_t e = fill_u32(cnt, 0u, M, s);
  if (e != hipSuccess) return e;
  k_block_groups<<<nblk(nb), kBlock, 0, s>>>(rows, skey, nb, X, R, cnt, first);
  e = scan_u32_to_u32(cnt, base, M, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_block_perm<<<nblk(nb), kBlock, 0, s>>>(rows, skey, nb, X, R, base, first, cnt, perm);
  return hipGetLastError();
}

hipError_t put_bodies(const Body* bodies, int32_t nb, Body* dst, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (nb > kBodyPack) return hipErrorInvalidValue;
  BodyPack p;
  std::memcpy(&p.b[0], bodies, sizeof(Body) * (size_t)nb);
  k_put_bodies<<<1, 256, 0, s>>>(p, nb, dst);
  return hipGetLastError();
}

hipError_t tile_tables(const int32_t* rows, int64_t rows_cap, const uint64_t* n_dev, const uint32_t* skey,
                       const uint32_t* cs, Phys P, uint32_t* tabs, hipStream_t s) {
  if (rows_cap <= 0) return hipSuccess;
  const int64_t nb = (rows_cap + kRows - 1) / kRows;
  k_tile_tables<<<nblk(nb), kBlock, 0, s>>>(rows, n_dev, skey, cs, P, tabs);
  return hipGetLastError();
}

hipError_t nbr_fill_soil(const int32_t* rows, int64_t n_rows, const float4* pos4, const int4* cpos,
                         const uint32_t* skey, const uint32_t* cs, Grid g, const uint32_t* cnt,
                         const uint32_t* stash, const uint64_t* off, uint32_t* nbr, const uint32_t* tabs,
                         uint16_t* tix, uint32_t skip_cap, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  k_nbr_fill_soil<<<soil_blocks(n_rows), kListBlock, 0, s>>>(rows, n_rows, pos4, cpos, skey, cs, g, cnt, stash, off, nbr,
                                                             tabs, tix, skip_cap);
  return hipGetLastError();
}

hipError_t nbr_slots(int64_t n_rows, const uint64_t* off, const uint32_t* tabs, const uint16_t* tix, uint32_t* nbr,
                     uint32_t skip_cap, hipStream_t s) {
  if (n_rows <= 0 || skip_cap == 0) return hipSuccess;
  k_nbr_slots<<<soil_blocks(n_rows), kListBlock, 0, s>>>(n_rows, off, tabs, tix, nbr, skip_cap);
  return hipGetLastError();
}

uint32_t tile_records(int cfg, bool cell) {
  if (cfg == 1) return cell ? tile_cap<true, 1>() : tile_cap<false, 1>();
  if (cfg == 2) return cell ? tile_cap<true, 2>() : tile_cap<false, 2>();
  return 0;
}

int64_t tile_table_words(int64_t rows_cap) { return ((rows_cap + kRows - 1) / kRows + 1) * kTabWords; }

template <int CFG>
void launch_stage1(CPlanes A, Planes B, const int32_t* rows, int64_t n, const uint64_t* off, const uint32_t* nbr,
                   const Phys& P, const StageTape& T, bool tape, const uint32_t* tabs, const uint16_t* tix,
                   hipStream_t s) {
  const unsigned g = soil_blocks(n);
  if (P.cell) {
    if (tape) k_fluid_stage1<true, true, CFG><<<g, kStageBlock, 0, s>>>(A, B, rows, n, off, nbr, P, T, tabs, tix);
    else k_fluid_stage1<true, false, CFG><<<g, kStageBlock, 0, s>>>(A, B, rows, n, off, nbr, P, T, tabs, tix);
  } else {
    if (tape) k_fluid_stage1<false, true, CFG><<<g, kStageBlock, 0, s>>>(A, B, rows, n, off, nbr, P, T, tabs, tix);
    else k_fluid_stage1<false, false, CFG><<<g, kStageBlock, 0, s>>>(A, B, rows, n, off, nbr, P, T, tabs, tix);
  }
}

template <int CFG>
void launch_stage2(CPlanes B, Planes A, const int32_t* rows, int64_t n, const uint64_t* off, const uint32_t* nbr,
                   const Phys& P, const StageTape& T, bool tape, const uint32_t* tabs, const uint16_t* tix,
                   hipStream_t s) {
  const unsigned g = soil_blocks(n);
  if (P.cell) {
    if (tape) k_fluid_stage2<true, true, CFG><<<g, kStageBlock, 0, s>>>(B, A, rows, n, off, nbr, P, T, tabs, tix);
    else k_fluid_stage2<true, false, CFG><<<g, kStageBlock, 0, s>>>(B, A, rows, n, off, nbr, P, T, tabs, tix);
  } else {
    if (tape) k_fluid_stage2<false, true, CFG><<<g, kStageBlock, 0, s>>>(B, A, rows, n, off, nbr, P, T, tabs, tix);
    else k_fluid_stage2<false, false, CFG><<<g, kStageBlock, 0, s>>>(B, A, rows, n, off, nbr, P, T, tabs, tix);
  }
}

hipError_t fluid_stage1(CPlanes A, Planes B, const int32_t* rows, int64_t n, const uint64_t* off,
                        const uint32_t* nbr, Phys P, const StageTape* tape, const uint32_t* tabs,
                        const uint16_t* tix, int cfg, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const StageTape T = tape ? *tape : StageTape{};
  if (cfg == 0) launch_stage1<0>(A, B, rows, n, off, nbr, P, T, tape != nullptr, tabs, tix, s);
  else if (cfg == 1) launch_stage1<1>(A, B, rows, n, off, nbr, P, T, tape != nullptr, tabs, tix, s);
  else launch_stage1<2>(A, B, rows, n, off, nbr, P, T, tape != nullptr, tabs, tix, s);
  return hipGetLastError();
}

hipError_t fluid_stage2(CPlanes B, Planes A, const int32_t* rows, int64_t n, const uint64_t* off,
                        const uint32_t* nbr, Phys P, const StageTape* tape, const uint32_t* tabs,
                        const uint16_t* tix, int cfg, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const StageTape T = tape ? *tape : StageTape{};
  if (cfg == 0) launch_stage2<0>(B, A, rows, n, off, nbr, P, T, tape != nullptr, tabs, tix, s);
  else if (cfg == 1) launch_stage2<1>(B, A, rows, n, off, nbr, P, T, tape != nullptr, tabs, tix, s);
  else launch_stage2<2>(B, A, rows, n, off, nbr, P, T, tape != nullptr, tabs, tix, s);
  return hipGetLastError();
}

hipError_t scatter_rows(CPlanes src, const int32_t* rows, int64_t n, const int32_t* slot_id, float4* m_a,
                        float4* m_b, float4* m_c, float4* m_d, uint32_t* key, bool cell, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_scatter<<<nblk(n), kBlock, 0, s>>>(src, rows, n, slot_id, m_a, m_b, m_c, m_d, key, cell ? 1 : 0);
  return hipGetLastError();
}

hipError_t key_fill(const float4* m_a, const float4* m_d, int64_t n, bool cell, uint32_t* key, hipStream_t s) {
  if (n <= 0 || !key) return hipSuccess;
  k_key_fill<<<nblk(n), kBlock, 0, s>>>(m_a, m_d, n, cell ? 1 : 0, key);
  return hipGetLastError();
}

hipError_t scatter_marker_rows(CPlanes src, const int32_t* rows, int64_t n, const int32_t* slot_id, float4* m_b,
                               float4* m_c, float4* m_d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_scatter_markers<<<nblk(n), kBlock, 0, s>>>(src, rows, n, slot_id, m_b, m_c, m_d);
  return hipGetLastError();
}

// ------------------------------------------------------ static scratch ---
// Scratch of the step that allocates nothing: scan tile totals, compaction
// block counts and the chunk sums of the body-force reduction, carved from one
// file-scope array. Every device the library runs on holds its own copy until
// the process ends; in host code the array's name is not a device address, so
// each device's address is looked up once (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (!out || device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    addr[device] = ptr;
  }
  *out = addr[device];
  return hipSuccess;
}

}  // namespace crm
