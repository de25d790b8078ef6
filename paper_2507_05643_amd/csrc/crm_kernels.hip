// HIP kernels of the CRM particle step for gfx950 (CDNA4, wave64).
//
// Paper: arXiv 2507.05643 (Chrono::CRM). Sections cited per kernel.
// Nothing here is a dense contraction, so no MFMA: the neighbour interaction
// is FP32 VALU work over cell-sorted records, the binning/compaction steps are
// HBM streams built from wave64 ballots and block scans.
#include "crm_internal.h"

namespace crm {
namespace {

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ inline int wave_id() { return threadIdx.x / kWave; }
__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// The dispatcher hands workgroup b to XCD b % 8, and each XCD has its own L2.
// Neighbouring particles are neighbours in the cell-sorted order, so give
// every XCD one contiguous range of logical blocks: XCD x gets
// [x q + min(x, r), ...) of length q + (x < r), with q, r = nblocks / 8, % 8.
// This is a bijection of [0, nblocks).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t q = nb / kXcds, r = nb % kXcds;
  const int64_t x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}

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

template <typename TOut>
__global__ __launch_bounds__(kBlock) void k_scan_top(TOut* __restrict__ bsum, int64_t nb,
                                                     TOut* __restrict__ out_total) {
  TOut carry = 0;
  for (int64_t base = 0; base < nb; base += kBlock) {
    int64_t i = base + threadIdx.x;
    TOut v = (i < nb) ? bsum[i] : TOut(0);
    TOut tot;
    TOut ex = block_excl_scan(v, tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *out_total = carry;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const TIn* __restrict__ in, int64_t n,
                                                       const TOut* __restrict__ boff,
                                                       TOut* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TOut carry = boff[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    TOut v = (i < n) ? (TOut)in[i] : TOut(0);
    TOut tot;
    TOut ex = block_excl_scan(v, tot);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
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
  k_scan_top<TOut><<<1, kBlock, 0, s>>>(tmp, nb, out + n);
  k_scan_apply<TIn, TOut><<<(unsigned)nb, kBlock, 0, s>>>(in, n, tmp, out);
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
                                                       int32_t* __restrict__ out) {
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

__global__ void k_copy2(uint64_t* dst, const uint64_t* a, const uint64_t* b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = *a;
    dst[1] = *b;
  }
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
  k_pred_write<Pred><<<(unsigned)nb, kBlock, 0, s>>>(pr, n, boff, out);
  k_store_count<<<1, 64, 0, s>>>(count_dst, boff + nb);
  return hipGetLastError();
}

// ------------------------------------------------------ exact FP64 helpers ---
// These reproduce, operation by operation, the FP64 arithmetic that decides
// integers (cells, neighbour membership, activity flags, marker placement), so
// that they do not depend on FMA contraction.
__device__ inline int32_t cell_coord(double x, double lo, double inv, int32_t dim) {
#pragma clang fp contract(off)
  double t = floor((x - lo) * inv);
  if (!(t >= 0.0)) return 0;
  if (t > (double)(dim - 1)) return dim - 1;
  return (int32_t)t;
}

__device__ inline double dist2_fp64(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
  double dx = (double)ax - (double)bx;
  double dy = (double)ay - (double)by;
  double dz = (double)az - (double)bz;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ inline void body_point(const Body& b, float lx, float ly, float lz, double out[3]) {
#pragma clang fp contract(off)
  double l0 = lx, l1 = ly, l2 = lz;
  for (int a = 0; a < 3; ++a)
    out[a] = b.X[a] + ((b.R[3 * a] * l0 + b.R[3 * a + 1] * l1) + b.R[3 * a + 2] * l2);
}

// ---------------------------------------------------- markers and flags ---
__global__ __launch_bounds__(kBlock) void k_place_markers_master(const float4* __restrict__ local, int64_t nm,
                                                                 int64_t n_soil, const Body* __restrict__ bodies,
                                                                 float4* __restrict__ m_a) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= nm) return;
  float4 l = local[k];
  const Body& b = bodies[__float_as_uint(l.w)];
  double x[3];
  body_point(b, l.x, l.y, l.z, x);
  float4 o = m_a[n_soil + k];
  o.x = (float)x[0];
  o.y = (float)x[1];
  o.z = (float)x[2];
  m_a[n_soil + k] = o;
}

// Sec. 4.2 item 2: Active inside an oriented box (|R^T (x - X)| <= half per
// local axis), Extended-Active inside the box grown by 2h, else Inactive.
__global__ __launch_bounds__(kBlock) void k_activity(const float4* __restrict__ m_a, int64_t n,
                                                     const Body* __restrict__ bodies, int32_t nb, Grid g,
                                                     uint8_t* __restrict__ flags) {
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float4 p = m_a[i];
  double xw[3] = {(double)p.x, (double)p.y, (double)p.z};
  uint8_t best = 0;
  for (int b = 0; b < nb; ++b) {
    const Body& B = bodies[b];
    if (!B.has_box) continue;
    double d[3], l[3];
    for (int a = 0; a < 3; ++a) d[a] = xw[a] - B.X[a];
    for (int a = 0; a < 3; ++a) l[a] = (B.R[a] * d[0] + B.R[3 + a] * d[1]) + B.R[6 + a] * d[2];
    bool in = true, ext = true;
    for (int a = 0; a < 3; ++a) {
      double al = fabs(l[a]);
      if (!(al <= B.half[a])) in = false;
      if (!(al <= B.half[a] + g.ext)) ext = false;
    }
    if (in) { best = 2; break; }
    if (ext) best = 1;
  }
  flags[i] = best;
}

// ------------------------------------------------------ hashing and sort ---
// Sec. 4.1 step 1: c = z * (Y * X) + y * X + x with cell size 2h. The arrival
// rank of each particle in its cell comes from an atomic counter (counting sort).
__global__ __launch_bounds__(kBlock) void k_hash_count(const int32_t* __restrict__ ids, int64_t n,
                                                       const float4* __restrict__ m_a, Grid g,
                                                       uint32_t* __restrict__ key, uint32_t* __restrict__ rank,
                                                       uint32_t* __restrict__ cnt) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  int64_t id = ids ? ids[k] : k;
  float4 p = m_a[id];
  int32_t cx = cell_coord((double)p.x, g.lo[0], g.inv, g.dims[0]);
  int32_t cy = cell_coord((double)p.y, g.lo[1], g.inv, g.dims[1]);
  int32_t cz = cell_coord((double)p.z, g.lo[2], g.inv, g.dims[2]);
  uint32_t c = ((uint32_t)cz * (uint32_t)g.dims[1] + (uint32_t)cy) * (uint32_t)g.dims[0] + (uint32_t)cx;
  key[k] = c;
  rank[k] = atomicAdd(&cnt[c], 1u);
}

__global__ __launch_bounds__(kBlock) void k_place(const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
                                                  const uint32_t* __restrict__ cs, int64_t n,
                                                  uint32_t* __restrict__ tmp) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  tmp[cs[key[k]] + rank[k]] = (uint32_t)k;
}

// Sec. 4.1 step 2 (sort by cell, ties by particle id): the atomic arrival order
// inside a cell is replaced by the id order (a cell holds ~10-20 particles), and
// the master state is gathered into the cell-sorted working records.
__global__ __launch_bounds__(kBlock) void k_gather_sorted(
    const uint32_t* __restrict__ tmp, const uint32_t* __restrict__ key, const int32_t* __restrict__ ids,
    const uint32_t* __restrict__ cs, int64_t n, int64_t n_soil, const uint8_t* __restrict__ flags,
    const float4* __restrict__ m_a, const float4* __restrict__ m_b, const float4* __restrict__ m_c,
    const float4* __restrict__ m_d, Rec* __restrict__ A, Rec* __restrict__ B, float4* __restrict__ pos4,
    int32_t* __restrict__ slot_id, uint32_t* __restrict__ skey) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  uint32_t k = tmp[p];
  uint32_t c = key[k];
  uint32_t lo = cs[c], hi = cs[c + 1];
  uint32_t r = 0;
  for (uint32_t q = lo; q < hi; ++q) r += (tmp[q] < k) ? 1u : 0u;   // ids ascend with k
  uint32_t f = lo + r;
  int64_t id = ids ? ids[k] : (int64_t)k;
  slot_id[f] = (int32_t)id;
  skey[f] = c;
  Rec rec;
  rec.a = m_a[id];
  rec.b = m_b[id];
  rec.c = m_c[id];
  rec.d = m_d[id];
  uint32_t aux = __float_as_uint(rec.b.w) & ~3u;
  uint32_t kind = (id < n_soil) ? ((flags == nullptr || flags[id] == 2) ? kSoilActive : kSoilExtended) : kMarker;
  rec.b.w = __uint_as_float(aux | kind);
  A[f] = rec;
  B[f] = rec;
  pos4[f] = make_float4(rec.a.x, rec.a.y, rec.a.z, rec.b.w);
}

// ------------------------------------------------------- neighbour lists ---
// Algorithm 1: for each row particle, the 27 cells around its own; the three
// cells x-1..x+1 of a (y, z) row are consecutive in the sorted order, so they
// are scanned as one range [cellStart[c(x-1)], cellStart[c(x+1) + 1]).
// Membership |x_i - x_j| < 2h is decided in FP64 on the FP32 positions.
// With soil_only (marker rows) only soil candidates are kept: the BCE sums
// of Sec. 2.5.1 run over soil particles, so marker-marker pairs are never used.
template <bool FILL, typename Out>
__device__ inline uint32_t scan_neighbours(float4 pi, uint32_t c, const float4* __restrict__ pos4,
                                           const uint32_t* __restrict__ cs, const Grid& g, bool soil_only,
                                           Out out) {
  const int X = g.dims[0], Y = g.dims[1], Z = g.dims[2];
  const int cx = (int)(c % (uint32_t)X);
  const uint32_t t = c / (uint32_t)X;
  const int cy = (int)(t % (uint32_t)Y);
  const int cz = (int)(t / (uint32_t)Y);
  const int x0 = cx > 0 ? cx - 1 : 0;
  const int x1 = cx < X - 1 ? cx + 1 : X - 1;
  uint32_t count = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= Z) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= Y) continue;
      const uint32_t row = ((uint32_t)z * (uint32_t)Y + (uint32_t)y) * (uint32_t)X;
      const uint32_t b = cs[row + x0], e = cs[row + x1 + 1];
      for (uint32_t j = b; j < e; ++j) {
        float4 pj = pos4[j];
        if (soil_only && (__float_as_uint(pj.w) & 3u) == kMarker) continue;
        if (dist2_fp64(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z) < g.R2) {
          if (FILL) out[(size_t)count * kWave] = j;
          ++count;
        }
      }
    }
  }
  return count;
}

__global__ __launch_bounds__(kBlock) void k_nbr_count(const int32_t* __restrict__ rows, int64_t rows_cap,
                                                      const uint64_t* __restrict__ n_rows_dev,
                                                      const float4* __restrict__ pos4, const uint32_t* __restrict__ skey,
                                                      const uint32_t* __restrict__ cs, Grid g, int soil_only,
                                                      uint32_t* __restrict__ cnt, uint32_t* __restrict__ wave_len) {
  const int64_t r = xcd_block() * kBlock + threadIdx.x;
  const int64_t nr = (int64_t)*n_rows_dev;
  uint32_t count = 0;
  if (r < nr) {
    const int32_t s = rows[r];
    count = scan_neighbours<false>(pos4[s], skey[s], pos4, cs, g, soil_only != 0, (uint32_t*)nullptr);
  }
  if (r < rows_cap) cnt[r] = count;
  uint32_t mx = count;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    uint32_t y = __shfl_xor(mx, o, kWave);
    mx = y > mx ? y : mx;
  }
  if (lane_id() == 0 && r < rows_cap) wave_len[r / kWave] = mx * (uint32_t)kWave;
}

// Each wave gathers its entries in LDS and writes them out as whole 256-byte
// rows (lanes finish their candidate loops at different times, so direct
// stores would reach L2 as partial lines); a wave whose longest list exceeds
// the LDS slots writes directly.
constexpr int kFillSlots = 72;

__global__ __launch_bounds__(kBlock) void k_nbr_fill(const int32_t* __restrict__ rows, int64_t n_rows,
                                                     const float4* __restrict__ pos4, const uint32_t* __restrict__ skey,
                                                     const uint32_t* __restrict__ cs, Grid g, int soil_only,
                                                     const uint64_t* __restrict__ woff, uint32_t* __restrict__ nbr) {
  __shared__ uint32_t buf[kBlock / kWave][kFillSlots * kWave];
  const int64_t r = xcd_block() * kBlock + threadIdx.x;
  const int64_t w = r / kWave;
  const int lane = lane_id();
  const bool wave_live = w * kWave < n_rows;
  uint64_t base = 0;
  uint32_t wmax = 0;
  if (wave_live) {
    base = woff[w];
    wmax = (uint32_t)((woff[w + 1] - base) / kWave);
  }
  const bool use_lds = wmax <= (uint32_t)kFillSlots;
  uint32_t* lbuf = &buf[wave_id()][lane];
  if (r < n_rows) {
    const int32_t s = rows[r];
    if (use_lds)
      scan_neighbours<true>(pos4[s], skey[s], pos4, cs, g, soil_only != 0, lbuf);
    else
      scan_neighbours<true>(pos4[s], skey[s], pos4, cs, g, soil_only != 0, nbr + base + lane);
  }
  __syncthreads();
  if (wave_live && use_lds)
    for (uint32_t k = 0; k < wmax; ++k) nbr[base + (uint64_t)k * kWave + lane] = lbuf[k * kWave];
}

// ------------------------------------------------------- SPH kernel (FP32) ---
// Cubic spline with support 2h (Sec. 4.1): W = kw w(q) and
// grad_i W_ij = kf f(q) (x_i - x_j), f = W'(r) / (r h^-5 pi^-1 ...) folded so that
// the self pair (r = 0) gives a zero gradient without a division by r.
__device__ inline float kernel_f(float q, float kf) {
  if (q < 1.0f) return kf * (2.25f * q - 3.0f);
  if (q < 2.0f) {
    float t = 2.0f - q;
    return -0.75f * kf * t * t * __builtin_amdgcn_rcpf(q);
  }
  return 0.0f;
}

__device__ inline float kernel_w(float q, float kw) {
  if (q < 1.0f) return kw * (1.0f + q * q * (0.75f * q - 1.5f));
  if (q < 2.0f) {
    float t = 2.0f - q;
    return 0.25f * kw * t * t * t;
  }
  return 0.0f;
}

__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ------------------------------------------------------------ markers ---
__global__ __launch_bounds__(kBlock) void k_place_markers_working(const int32_t* __restrict__ mrows, int64_t n,
                                                                  const int32_t* __restrict__ slot_id, int64_t n_soil,
                                                                  const float4* __restrict__ local,
                                                                  const Body* __restrict__ bodies,
                                                                  Rec* __restrict__ A, Rec* __restrict__ B) {
  int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  int32_t s = mrows[r];
  float4 l = local[slot_id[s] - n_soil];
  double x[3];
  body_point(bodies[__float_as_uint(l.w)], l.x, l.y, l.z, x);
  float4 a = A[s].a;
  a.x = (float)x[0];
  a.y = (float)x[1];
  a.z = (float)x[2];
  A[s].a = a;
  B[s].a = a;
}

// Sec. 2.5.1: Adami velocity u~ = sum u_f W / sum W, no-slip u_s = 2 u_body - u~;
// stress s_s = [sum s_f W - ((g - a_s) . sum rho_f (x_s - x_f) W) I] / sum W.
// With `partials`, the marker acceleration from the momentum equation over the
// fluid neighbours (no body force) and the per-block body force and torque.
template <bool FORCE>
__global__ __launch_bounds__(kBlock) void k_bce(Rec* __restrict__ S, const int32_t* __restrict__ mrows, int64_t n,
                                                const uint32_t* __restrict__ cnt, const uint64_t* __restrict__ woff,
                                                const uint32_t* __restrict__ nbr, const Body* __restrict__ bodies,
                                                int32_t nb, Phys P, double* __restrict__ partials) {
  const int64_t r = xcd_block() * kBlock + threadIdx.x;
  const bool valid = r < n;
  int body = -1;
  double fr[6] = {0, 0, 0, 0, 0, 0};
  if (valid) {
    const int32_t s = mrows[r];
    Rec me = S[s];
    body = (int)(__float_as_uint(me.b.w) >> 2);
    const Body& B = bodies[body];
    const float xs = me.a.x, ys = me.a.y, zs = me.a.z;
    // body velocity and acceleration at the marker (FP64 lever arm)
    double rv[3] = {(double)xs - B.X[0], (double)ys - B.X[1], (double)zs - B.X[2]};
    double wr[3] = {B.W[1] * rv[2] - B.W[2] * rv[1], B.W[2] * rv[0] - B.W[0] * rv[2],
                    B.W[0] * rv[1] - B.W[1] * rv[0]};
    double wwr[3] = {B.W[1] * wr[2] - B.W[2] * wr[1], B.W[2] * wr[0] - B.W[0] * wr[2],
                     B.W[0] * wr[1] - B.W[1] * wr[0]};
    float ub[3], as[3];
    for (int a = 0; a < 3; ++a) ub[a] = (float)(B.V[a] + wr[a]);
    if (B.has_acc) {
      double ar[3] = {B.Al[1] * rv[2] - B.Al[2] * rv[1], B.Al[2] * rv[0] - B.Al[0] * rv[2],
                      B.Al[0] * rv[1] - B.Al[1] * rv[0]};
      for (int a = 0; a < 3; ++a) as[a] = (float)(B.A[a] + ar[a] + wwr[a]);
    } else {
      for (int a = 0; a < 3; ++a) as[a] = (float)wwr[a];
    }
    const uint32_t c = cnt[r];
    const uint32_t* lp = nbr + woff[r / kWave] + (r % kWave);
    float sw = 0.f, su0 = 0.f, su1 = 0.f, su2 = 0.f;
    float ss0 = 0.f, ss1 = 0.f, ss2 = 0.f, ss3 = 0.f, ss4 = 0.f, ss5 = 0.f;
    float sr0 = 0.f, sr1 = 0.f, sr2 = 0.f;
    for (uint32_t k = 0; k < c; ++k) {
      const uint32_t j = lp[(size_t)k * kWave];
      const Rec o = S[j];
      if ((__float_as_uint(o.b.w) & 3u) == kMarker) continue;
      const float dx = xs - o.a.x, dy = ys - o.a.y, dz = zs - o.a.z;
      const float q = fsqrt(dx * dx + dy * dy + dz * dz) * P.inv_h;
      const float w = kernel_w(q, P.kw);
      sw += w;
      su0 += o.b.x * w; su1 += o.b.y * w; su2 += o.b.z * w;
      ss0 += o.c.x * w; ss1 += o.c.y * w; ss2 += o.c.z * w;
      ss3 += o.c.w * w; ss4 += o.d.x * w; ss5 += o.d.y * w;
      const float rw = o.a.w * w;
      sr0 += rw * dx; sr1 += rw * dy; sr2 += rw * dz;
    }
    float us[3], sg[6];
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
      for (int a = 0; a < 6; ++a) sg[a] = 0.f;
    }
    me.b.x = us[0]; me.b.y = us[1]; me.b.z = us[2];
    me.c = make_float4(sg[0], sg[1], sg[2], sg[3]);
    me.d.x = sg[4]; me.d.y = sg[5];
    S[s].b = me.b;
    S[s].c = me.c;
    S[s].d = me.d;
    if (FORCE) {
      // Momentum equation at the marker (F3) with artificial viscosity,
      // fluid neighbours only: a_s = (1/rho_s) sum V_f (s_s + s_f) gradW + Pi.
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, v0 = 0.f, v1 = 0.f, v2 = 0.f;
      const float rhos = me.a.w;
      for (uint32_t k = 0; k < c; ++k) {
        const uint32_t j = lp[(size_t)k * kWave];
        const Rec o = S[j];
        if ((__float_as_uint(o.b.w) & 3u) == kMarker) continue;
        const float dx = xs - o.a.x, dy = ys - o.a.y, dz = zs - o.a.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float q = fsqrt(r2) * P.inv_h;
        const float F = kernel_f(q, P.kf);
        const float VF = P.m * __builtin_amdgcn_rcpf(o.a.w) * F;
        const float wx = VF * dx, wy = VF * dy, wz = VF * dz;
        const float sxx = sg[0] + o.c.x, syy = sg[1] + o.c.y, szz = sg[2] + o.c.z;
        const float sxy = sg[3] + o.c.w, sxz = sg[4] + o.d.x, syz = sg[5] + o.d.y;
        a0 += sxx * wx + sxy * wy + sxz * wz;
        a1 += sxy * wx + syy * wy + syz * wz;
        a2 += sxz * wx + syz * wy + szz * wz;
        if (P.av_mode != 0) {
          const float vr = (us[0] - o.b.x) * dx + (us[1] - o.b.y) * dy + (us[2] - o.b.z) * dz;
          if (P.av_mode == 1 || vr < 0.f) {
            const float cf = P.av_coef * vr * F *
                             __builtin_amdgcn_rcpf(0.5f * (rhos + o.a.w) * (r2 + P.xi2));
            v0 += cf * dx; v1 += cf * dy; v2 += cf * dz;
          }
        }
      }
      const float ir = 1.0f / rhos;
      const double f0 = (double)P.m * (double)(a0 * ir + v0);
      const double f1 = (double)P.m * (double)(a1 * ir + v1);
      const double f2 = (double)P.m * (double)(a2 * ir + v2);
      fr[0] = f0; fr[1] = f1; fr[2] = f2;
      fr[3] = rv[1] * f2 - rv[2] * f1;
      fr[4] = rv[2] * f0 - rv[0] * f2;
      fr[5] = rv[0] * f1 - rv[1] * f0;
    }
  }
  if (FORCE) {
    // Deterministic per-block sums per body (fixed tree order, no float atomics).
    __shared__ double red[6][kBlock];
    const int t = threadIdx.x;
    for (int b = 0; b < nb; ++b) {
      const int any = __syncthreads_or(body == b);
      if (!any) {
        if (t < 6) partials[(xcd_block() * nb + b) * 6 + t] = 0.0;
        continue;
      }
      for (int a = 0; a < 6; ++a) red[a][t] = (body == b) ? fr[a] : 0.0;
      __syncthreads();
      for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (t < o)
          for (int a = 0; a < 6; ++a) red[a][t] += red[a][t + o];
        __syncthreads();
      }
      if (t < 6) partials[(xcd_block() * nb + b) * 6 + t] = red[t][0];
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_body_reduce(const double* __restrict__ partials, int64_t nblocks,
                                                        int32_t nb, double* __restrict__ forces) {
  __shared__ double red[6][kBlock];
  const int b = blockIdx.x, t = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = t; k < nblocks; k += kBlock)
    for (int a = 0; a < 6; ++a) acc[a] += partials[(k * nb + b) * 6 + a];
  for (int a = 0; a < 6; ++a) red[a][t] = acc[a];
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (t < o)
      for (int a = 0; a < 6; ++a) red[a][t] += red[a][t + o];
    __syncthreads();
  }
  if (t < 6) forces[b * 6 + t] = red[t][0];
}

// ------------------------------------------------------------- fluid ---
struct Rates {
  float dx, dy, dz;           // position rate = own velocity
  float ax, ay, az;           // acceleration
  float s0, s1, s2, s3, s4, s5;  // stress rate
  float drho;
};

// Sec. 2.2: L = sum_j V_j (u_j - u_i) (x) gradW (F2); drho/dt = -rho tr L;
// a = (1/rho_i) sum_j V_j (s_i + s_j) . gradW + g + Pi_a (F3, artificial viscosity
// with the sign that repels approaching pairs); ds/dt = Om s - s Om + 2G D +
// (bulk K - 2G/3) tr D I with D, Om the symmetric and skew parts of L.
__device__ inline Rates fluid_rhs(const Rec& me, const Rec* __restrict__ S, uint32_t c,
                                  const uint32_t* __restrict__ lp, const Phys& P) {
  const float xi = me.a.x, yi = me.a.y, zi = me.a.z, rhoi = me.a.w;
  const float ux = me.b.x, uy = me.b.y, uz = me.b.z;
  const float s0 = me.c.x, s1 = me.c.y, s2 = me.c.z, s3 = me.c.w, s4 = me.d.x, s5 = me.d.y;
  float L00 = 0.f, L01 = 0.f, L02 = 0.f, L10 = 0.f, L11 = 0.f, L12 = 0.f, L20 = 0.f, L21 = 0.f, L22 = 0.f;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, v0 = 0.f, v1 = 0.f, v2 = 0.f;
  for (uint32_t k = 0; k < c; ++k) {
    const uint32_t j = lp[(size_t)k * kWave];
    const Rec o = S[j];
    const float dx = xi - o.a.x, dy = yi - o.a.y, dz = zi - o.a.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float q = fsqrt(r2) * P.inv_h;
    const float F = kernel_f(q, P.kf);
    const float VF = P.m * __builtin_amdgcn_rcpf(o.a.w) * F;   // V_j * (gradW / r_ij)
    const float wx = VF * dx, wy = VF * dy, wz = VF * dz;      // V_j grad_i W_ij
    const float dux = o.b.x - ux, duy = o.b.y - uy, duz = o.b.z - uz;
    L00 += dux * wx; L01 += dux * wy; L02 += dux * wz;
    L10 += duy * wx; L11 += duy * wy; L12 += duy * wz;
    L20 += duz * wx; L21 += duz * wy; L22 += duz * wz;
    const float sxx = s0 + o.c.x, syy = s1 + o.c.y, szz = s2 + o.c.z;
    const float sxy = s3 + o.c.w, sxz = s4 + o.d.x, syz = s5 + o.d.y;
    a0 += sxx * wx + sxy * wy + sxz * wz;
    a1 += sxy * wx + syy * wy + syz * wz;
    a2 += sxz * wx + syz * wy + szz * wz;
    if (P.av_mode != 0) {
      const float vr = -(dux * dx + duy * dy + duz * dz);      // v_ij . r_ij
      if (P.av_mode == 1 || vr < 0.f) {
        const float cf = P.av_coef * vr * F * __builtin_amdgcn_rcpf(0.5f * (rhoi + o.a.w) * (r2 + P.xi2));
        v0 += cf * dx; v1 += cf * dy; v2 += cf * dz;
      }
    }
  }
  Rates R;
  const float ir = 1.0f / rhoi;
  R.dx = ux; R.dy = uy; R.dz = uz;
  R.ax = a0 * ir + v0 + P.gx;
  R.ay = a1 * ir + v1 + P.gy;
  R.az = a2 * ir + v2 + P.gz;
  const float trD = L00 + L11 + L22;
  R.drho = -rhoi * trD;
  // spin components Om_xy, Om_xz, Om_yz and strain rate D
  const float wxy = 0.5f * (L01 - L10), wxz = 0.5f * (L02 - L20), wyz = 0.5f * (L12 - L21);
  const float Dxy = 0.5f * (L01 + L10), Dxz = 0.5f * (L02 + L20), Dyz = 0.5f * (L12 + L21);
  // M = Om s; Om s - s Om = M + M^T
  const float Mxx = wxy * s3 + wxz * s4;
  const float Myy = -wxy * s3 + wyz * s5;
  const float Mzz = -wxz * s4 - wyz * s5;
  const float Mxy = wxy * s1 + wxz * s5, Myx = -wxy * s0 + wyz * s4;
  const float Mxz = wxy * s5 + wxz * s2, Mzx = -wxz * s0 - wyz * s3;
  const float Myz = -wxy * s4 + wyz * s2, Mzy = -wxz * s3 - wyz * s1;
  const float iso = P.iso * trD;
  R.s0 = 2.f * Mxx + P.two_G * L00 + iso;
  R.s1 = 2.f * Myy + P.two_G * L11 + iso;
  R.s2 = 2.f * Mzz + P.two_G * L22 + iso;
  R.s3 = Mxy + Myx + P.two_G * Dxy;
  R.s4 = Mxz + Mzx + P.two_G * Dxz;
  R.s5 = Myz + Mzy + P.two_G * Dyz;
  return R;
}

__device__ inline void p_taubar(const float s[6], float& p, float& tb) {
  p = -(s[0] + s[1] + s[2]) * (1.0f / 3.0f);
  const float t0 = s[0] + p, t1 = s[1] + p, t2 = s[2] + p;
  tb = fsqrt(0.5f * (t0 * t0 + t1 * t1 + t2 * t2 + 2.f * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5])));
}

// Sec. 2.4: four-step return mapping of the trial stress st with taubar^n from sn.
__device__ inline void return_map(float st[6], const float sn[6], const Phys& P) {
  float ps, tbs, pn, tbn;
  p_taubar(st, ps, tbs);
  if (ps < P.p_cri) {
    for (int a = 0; a < 6; ++a) st[a] = 0.f;
    return;
  }
  p_taubar(sn, pn, tbn);
  float gd = (tbs - tbn) * P.inv_Gdt;
  float mu;
  if (!(gd > 0.f)) {
    mu = P.mu_s;
  } else if (ps <= 0.f) {
    mu = P.mu_2;
  } else {
    const float I = gd * P.grain_d * fsqrt(P.rho0 / ps);
    mu = P.mu_s + (P.mu_2 - P.mu_s) / (1.0f + P.I0 / I);
  }
  float tmax = mu * ps + P.cohesion;
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

// Stage 1 of the explicit midpoint rule (Sec. 2.3): B = A + dt/2 f(A).
__global__ __launch_bounds__(kBlock) void k_fluid_stage1(const Rec* __restrict__ A, Rec* __restrict__ B,
                                                         const int32_t* __restrict__ rows, int64_t n,
                                                         const uint32_t* __restrict__ cnt,
                                                         const uint64_t* __restrict__ woff,
                                                         const uint32_t* __restrict__ nbr, Phys P) {
  const int64_t r = xcd_block() * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const Rec me = A[s];
  const Rates R = fluid_rhs(me, A, cnt[r], nbr + woff[r / kWave] + (r % kWave), P);
  const float h = P.half_dt;
  Rec o;
  o.a = make_float4(me.a.x + h * R.dx, me.a.y + h * R.dy, me.a.z + h * R.dz, me.a.w + h * R.drho);
  o.b = make_float4(me.b.x + h * R.ax, me.b.y + h * R.ay, me.b.z + h * R.az, me.b.w);
  o.c = make_float4(me.c.x + h * R.s0, me.c.y + h * R.s1, me.c.z + h * R.s2, me.c.w + h * R.s3);
  o.d = make_float4(me.d.x + h * R.s4, me.d.y + h * R.s5, me.d.z, me.d.w);
  B[s] = o;
}

// Stage 2: A = A + dt f(B), then the return mapping on the stress.
__global__ __launch_bounds__(kBlock) void k_fluid_stage2(const Rec* __restrict__ B, Rec* __restrict__ A,
                                                         const int32_t* __restrict__ rows, int64_t n,
                                                         const uint32_t* __restrict__ cnt,
                                                         const uint64_t* __restrict__ woff,
                                                         const uint32_t* __restrict__ nbr, Phys P) {
  const int64_t r = xcd_block() * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const Rec mid = B[s];
  const Rates R = fluid_rhs(mid, B, cnt[r], nbr + woff[r / kWave] + (r % kWave), P);
  const Rec y = A[s];
  const float h = P.dt;
  float sn[6] = {y.c.x, y.c.y, y.c.z, y.c.w, y.d.x, y.d.y};
  float st[6] = {sn[0] + h * R.s0, sn[1] + h * R.s1, sn[2] + h * R.s2,
                 sn[3] + h * R.s3, sn[4] + h * R.s4, sn[5] + h * R.s5};
  return_map(st, sn, P);
  Rec o;
  o.a = make_float4(y.a.x + h * R.dx, y.a.y + h * R.dy, y.a.z + h * R.dz, y.a.w + h * R.drho);
  o.b = make_float4(y.b.x + h * R.ax, y.b.y + h * R.ay, y.b.z + h * R.az, y.b.w);
  o.c = make_float4(st[0], st[1], st[2], st[3]);
  o.d = make_float4(st[4], st[5], y.d.z, y.d.w);
  A[s] = o;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const Rec* __restrict__ src, const int32_t* __restrict__ rows,
                                                    int64_t n, const int32_t* __restrict__ slot_id,
                                                    float4* __restrict__ m_a, float4* __restrict__ m_b,
                                                    float4* __restrict__ m_c, float4* __restrict__ m_d) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const int32_t id = slot_id[s];
  const Rec v = src[s];
  m_a[id] = v.a;
  m_b[id] = v.b;
  m_c[id] = v.c;
  m_d[id] = v.d;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

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

hipError_t place_markers_master(const float4* local, int64_t nm, int64_t n_soil, const Body* bodies,
                                float4* m_a, hipStream_t s) {
  if (nm <= 0) return hipSuccess;
  k_place_markers_master<<<nblk(nm), kBlock, 0, s>>>(local, nm, n_soil, bodies, m_a);
  return hipGetLastError();
}

hipError_t activity_flags(const float4* m_a, int64_t n, const Body* bodies, int32_t nb, Grid g,
                          uint8_t* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_activity<<<nblk(n), kBlock, 0, s>>>(m_a, n, bodies, nb, g, flags);
  return hipGetLastError();
}

size_t compact_tmp_elems(int64_t n) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  return (size_t)(2 * nb + 1) + scan_tmp_elems(nb);
}

hipError_t compact_flags(const uint8_t* flags, int64_t n, int32_t* out_ids, uint64_t* count_dst,
                         uint32_t* tmp, hipStream_t s) {
  return compact_impl(PredFlags{flags}, n, out_ids, count_dst, tmp, s);
}

hipError_t compact_kind(const float4* pos4, int64_t n, uint32_t kind, int32_t* rows, uint64_t* count_dst,
                        uint32_t* tmp, hipStream_t s) {
  return compact_impl(PredKind{pos4, kind}, n, rows, count_dst, tmp, s);
}

hipError_t hash_count(const int32_t* ids, int64_t n, const float4* m_a, Grid g, uint32_t* key,
                      uint32_t* rank, uint32_t* cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_hash_count<<<nblk(n), kBlock, 0, s>>>(ids, n, m_a, g, key, rank, cnt);
  return hipGetLastError();
}

hipError_t place_sorted(const uint32_t* key, const uint32_t* rank, const uint32_t* cs, int64_t n,
                        uint32_t* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_place<<<nblk(n), kBlock, 0, s>>>(key, rank, cs, n, tmp);
  return hipGetLastError();
}

hipError_t gather_sorted(const uint32_t* tmp, const uint32_t* key, const int32_t* ids, const uint32_t* cs,
                         int64_t n, int64_t n_soil, const uint8_t* flags, const float4* m_a,
                         const float4* m_b, const float4* m_c, const float4* m_d, Rec* A, Rec* B,
                         float4* pos4, int32_t* slot_id, uint32_t* skey, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_gather_sorted<<<nblk(n), kBlock, 0, s>>>(tmp, key, ids, cs, n, n_soil, flags, m_a, m_b, m_c, m_d, A, B,
                                             pos4, slot_id, skey);
  return hipGetLastError();
}

hipError_t nbr_count(const int32_t* rows, int64_t rows_cap, const uint64_t* n_rows_dev, const float4* pos4,
                     const uint32_t* skey, const uint32_t* cs, Grid g, bool soil_only, uint32_t* cnt,
                     uint32_t* wave_len, hipStream_t s) {
  if (rows_cap <= 0) return hipSuccess;
  k_nbr_count<<<nblk(rows_cap), kBlock, 0, s>>>(rows, rows_cap, n_rows_dev, pos4, skey, cs, g, soil_only ? 1 : 0,
                                                cnt, wave_len);
  return hipGetLastError();
}

hipError_t nbr_fill(const int32_t* rows, int64_t n_rows, const float4* pos4, const uint32_t* skey,
                    const uint32_t* cs, Grid g, bool soil_only, const uint64_t* woff, uint32_t* nbr, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  k_nbr_fill<<<nblk(n_rows), kBlock, 0, s>>>(rows, n_rows, pos4, skey, cs, g, soil_only ? 1 : 0, woff, nbr);
  return hipGetLastError();
}

hipError_t place_markers_working(const int32_t* mrows, int64_t n, const int32_t* slot_id, int64_t n_soil,
                                 const float4* local, const Body* bodies, Rec* A, Rec* B, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_place_markers_working<<<nblk(n), kBlock, 0, s>>>(mrows, n, slot_id, n_soil, local, bodies, A, B);
  return hipGetLastError();
}

int64_t bce_blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

hipError_t bce(Rec* S, const int32_t* mrows, int64_t n, const uint32_t* cnt, const uint64_t* woff,
               const uint32_t* nbr, const Body* bodies, int32_t nb, Phys P, double* partials, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (partials)
    k_bce<true><<<nblk(n), kBlock, 0, s>>>(S, mrows, n, cnt, woff, nbr, bodies, nb, P, partials);
  else
    k_bce<false><<<nblk(n), kBlock, 0, s>>>(S, mrows, n, cnt, woff, nbr, bodies, nb, P, nullptr);
  return hipGetLastError();
}

hipError_t body_reduce(const double* partials, int64_t nblocks, int32_t nb, double* forces, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  k_body_reduce<<<(unsigned)nb, kBlock, 0, s>>>(partials, nblocks, nb, forces);
  return hipGetLastError();
}

hipError_t fluid_stage1(const Rec* A, Rec* B, const int32_t* rows, int64_t n, const uint32_t* cnt,
                        const uint64_t* woff, const uint32_t* nbr, Phys P, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fluid_stage1<<<nblk(n), kBlock, 0, s>>>(A, B, rows, n, cnt, woff, nbr, P);
  return hipGetLastError();
}

hipError_t fluid_stage2(const Rec* B, Rec* A, const int32_t* rows, int64_t n, const uint32_t* cnt,
                        const uint64_t* woff, const uint32_t* nbr, Phys P, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fluid_stage2<<<nblk(n), kBlock, 0, s>>>(B, A, rows, n, cnt, woff, nbr, P);
  return hipGetLastError();
}

hipError_t scatter_rows(const Rec* src, const int32_t* rows, int64_t n, const int32_t* slot_id, float4* m_a,
                        float4* m_b, float4* m_c, float4* m_d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_scatter<<<nblk(n), kBlock, 0, s>>>(src, rows, n, slot_id, m_a, m_b, m_c, m_d);
  return hipGetLastError();
}

}  // namespace crm
