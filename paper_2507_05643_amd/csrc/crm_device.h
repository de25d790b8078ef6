// Device helpers shared by the step kernels (crm_kernels.hip) and the
// adjoint kernels (crm_adjoint.hip): lane groups, XCD-aware block order, exact
// FP64 position helpers, the FP32 SPH kernel and the neighbour walk.
#pragma once

#include "crm_internal.h"

namespace crm {

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ inline int wave_id() { return threadIdx.x / kWave; }
__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// The dispatcher hands workgroup b to XCD b % 8, and each XCD has its own L2.
// Neighbouring particles are neighbours in the cell-sorted order, so give
// every XCD one contiguous range of logical blocks: XCD x gets
// [x q + min(x, r), ...) of length q + (x < r), with q, r = nb / 8, % 8.
// This is a bijection of [0, nb); blocks from nb on keep their index (used
// when only the first nb blocks of a grid carry live rows).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block_n(int64_t nb) {
  const int64_t b = blockIdx.x;
  if (b >= nb) return b;
  const int64_t q = nb / kXcds, r = nb % kXcds;
  const int64_t x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}
__device__ inline int64_t xcd_block() { return xcd_block_n(gridDim.x); }

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

// FP64 position -> cell index + FP32 offset: c = floor((x - lo) / S), o = x - lo - c S.
__device__ inline void to_cell(double x, double lo, double inv, double S, int32_t& c, float& o) {
#pragma clang fp contract(off)
  const double t = x - lo;
  const double cc = floor(t * inv);
  c = (int32_t)cc;
  o = (float)(t - cc * S);
}

// Absolute FP64 coordinate of a cell-offset position: (lo + c S) + o.
__device__ inline double from_cell(int32_t c, float o, double lo, double S) {
#pragma clang fp contract(off)
  return (lo + (double)c * S) + (double)o;
}

// Stored position (a = offsets or coordinates, d.zw = cells) -> FP64 absolute.
__device__ inline void abs_pos(float4 a, float4 d, const Grid& g, double x[3]) {
  if (g.cell) {
    const uint32_t w = __float_as_uint(d.w);
    x[0] = from_cell((int32_t)__float_as_uint(d.z), a.x, g.lo[0], g.S);
    x[1] = from_cell(unpack_y(w), a.y, g.lo[1], g.S);
    x[2] = from_cell(unpack_z(w), a.z, g.lo[2], g.S);
  } else {
    x[0] = a.x;
    x[1] = a.y;
    x[2] = a.z;
  }
}

// FP64 world position -> stored position (a.xyz and, for cells, d.zw).
__device__ inline void store_pos(const double x[3], const Grid& g, float4& a, float4& d) {
  if (g.cell) {
    int32_t c[3];
    float o[3];
    for (int q = 0; q < 3; ++q) to_cell(x[q], g.lo[q], g.inv, g.S, c[q], o[q]);
    a.x = o[0];
    a.y = o[1];
    a.z = o[2];
    d.z = __uint_as_float((uint32_t)c[0]);
    d.w = __uint_as_float(pack_yz(c[1], c[2]));
  } else {
    a.x = (float)x[0];
    a.y = (float)x[1];
    a.z = (float)x[2];
  }
}


// --------------------------------------------------------- lane groups ---
// A row (a soil particle or a marker) is served by a group of G consecutive
// lanes: the group walks the row's candidates or neighbours G at a time, so
// that the lanes of a group touch consecutive slots of the cell-sorted planes,
// and then sums its partial results across the group. The list passes, the
// marker rows and the reverse sweep use groups of kGroup lanes; the soil
// stages use narrower groups (more rows per wave share the per-row work).
constexpr int kGroup = 8;
static_assert(kWave % kGroup == 0, "group must divide the wave");

template <int G = kGroup>
__device__ inline int group_lane() { return threadIdx.x & (G - 1); }

// Sum over the G lanes of a group; every lane gets the total. DPP lane
// permutations: swap neighbours, swap pairs, mirror the two quads of 8 lanes,
// mirror the two halves of 16 lanes.
template <int Ctrl>
__device__ inline float dpp_perm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xF, 0xF, false));
}
template <int G = kGroup>
__device__ inline float group_sum(float v) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group of 2, 4, 8 or 16 lanes");
  v += dpp_perm<0xB1>(v);                          // quad [1,0,3,2]
  if (G >= 4) v += dpp_perm<0x4E>(v);              // quad [2,3,0,1]
  if (G >= 8) v += dpp_perm<0x141>(v);             // half-row mirror
  if (G >= 16) v += dpp_perm<0x140>(v);            // row mirror
  return v;
}

// Bits of this lane's group in a wave ballot.
template <int G = kGroup>
__device__ inline uint32_t group_bits(uint64_t ballot) {
  return (uint32_t)(ballot >> (lane_id() & ~(G - 1))) & ((1u << G) - 1u);
}


// ------------------------------------------------------- SPH kernel (FP32) ---
// Cubic spline with support 2h (Sec. 4.1): W = kw w(q) and
// grad_i W_ij = kf f(q) (x_i - x_j) with f = h^5 pi W'(r) / r, so that the self
// pair (r = 0) gives a zero gradient without a division by r.
__device__ inline float kernel_f(float q, float kf) {
  const float t = fmaxf(2.0f - q, 0.0f);
  const float outer = -0.75f * kf * t * t * __builtin_amdgcn_rcpf(q);   // 1 <= q < 2 (0 beyond)
  const float inner = kf * (2.25f * q - 3.0f);                          // q < 1
  return q < 1.0f ? inner : outer;
}

__device__ inline float kernel_w(float q, float kw) {
  const float t = fmaxf(2.0f - q, 0.0f);
  const float outer = 0.25f * kw * t * t * t;
  const float inner = kw * (1.0f + q * q * (0.75f * q - 1.5f));
  return q < 1.0f ? inner : outer;
}

__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Quintic Wendland C2: W = kw t^4 (2q + 1) and W'(r) / r = -kf t^3, t = 1 - q/2
// (zero beyond q = 2).
__device__ inline float wendland_w(float q, float kw) {
  const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
  const float t2 = t * t;
  return kw * t2 * t2 * (2.0f * q + 1.0f);
}

__device__ inline float wendland_f(float q, float kf) {
  const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
  return -kf * t * t * t;
}

// The context's smoothing kernel (uniform over a launch).
__device__ inline float sph_w(float q, const Phys& P) {
  return P.kern == 1 ? wendland_w(q, P.kw) : kernel_w(q, P.kw);
}

__device__ inline float sph_f(float q, const Phys& P) {
  return P.kern == 1 ? wendland_f(q, P.kf) : kernel_f(q, P.kf);
}

// The same with 1 / q supplied (iq; only the cubic's outer piece uses it).
__device__ inline float sph_f_iq(float q, float iq, const Phys& P) {
  if (P.kern == 1) return wendland_f(q, P.kf);
  const float t = fmaxf(2.0f - q, 0.0f);
  const float outer = -0.75f * P.kf * t * t * iq;
  const float inner = P.kf * (2.25f * q - 3.0f);
  return q < 1.0f ? inner : outer;
}

// A neighbour's record, loaded from the four planes with a 32-bit byte offset
// from each plane's base (slots < 2^28).
struct Nbr {
  float4 a, b, c, d;
};

__device__ inline const float4& at(const float4* base, uint32_t j) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(base) + (j << 4));
}

__device__ inline Nbr load_nbr(const CPlanes& S, uint32_t j) {
  Nbr n;
  n.a = at(S.a, j);
  n.b = at(S.b, j);
  n.c = at(S.c, j);
  n.d = at(S.d, j);
  return n;
}

// Neighbour records read straight from the four planes in HBM (through L1/L2).
struct GlobalLoad {
  static constexpr bool kTile = false;
  CPlanes S;
  __device__ Nbr operator()(uint32_t j) const { return load_nbr(S, j); }
};

// Walks entries k0 + lane, k0 + lane + G, ... < k1 of a CSR row and calls
// f(record, slot) for each, in that order, with the record from `load`. Two
// entries per lane and step: both slots, then both records, are in flight
// together (the second pair of loads repeats the first past the row's end).
template <int G = kGroup, class Load, class Fn>
__device__ inline void walk_row_with(const Load& load, uint64_t k0, uint64_t k1, const uint32_t* __restrict__ nbr,
                                     Fn&& f) {
  for (uint64_t k = k0 + group_lane<G>(); k < k1; k += 2 * G) {
    const bool has1 = k + G < k1;
    const uint32_t j0 = nbr[k];
    const uint32_t j1 = nbr[has1 ? k + G : k];
    const Nbr a = load(j0);
    const Nbr b = load(j1);
    f(a, j0);
    if (has1) f(b, j1);
  }
}

template <int G = kGroup, class Fn>
__device__ inline void walk_row(const CPlanes& S, uint64_t k0, uint64_t k1, const uint32_t* __restrict__ nbr,
                                Fn&& f) {
  walk_row_with<G>(GlobalLoad{S}, k0, k1, nbr, f);
}

// Own position of a row for pair separations: coordinates (FP32 absolute) or
// offsets plus integer cell (cell-offset positions).
struct Own {
  float x, y, z;
  int32_t cx, cy, cz;
};

template <bool CELL>
__device__ inline Own own_pos(float4 a, float4 d) {
  Own p{a.x, a.y, a.z, 0, 0, 0};
  if (CELL) {
    const uint32_t w = __float_as_uint(d.w);
    p.cx = (int32_t)__float_as_uint(d.z);
    p.cy = unpack_y(w);
    p.cz = unpack_z(w);
  }
  return p;
}

// x_i - x_j in FP32: the coordinate difference, plus the cell difference times
// the cell size for cell-offset positions.
template <bool CELL>
__device__ inline void pair_sep(const Own& p, const Nbr& o, float Sf, float& dx, float& dy, float& dz) {
  dx = p.x - o.a.x;
  dy = p.y - o.a.y;
  dz = p.z - o.a.z;
  if (CELL) {
    const uint32_t w = __float_as_uint(o.d.w);
    dx += (float)(p.cx - (int32_t)__float_as_uint(o.d.z)) * Sf;
    dy += (float)(p.cy - unpack_y(w)) * Sf;
    dz += (float)(p.cz - unpack_z(w)) * Sf;
  }
}

// x + h u for one stored position: FP32 for absolute coordinates; for
// cell-offset positions the offset is advanced in FP64 and folded back into
// [0, S) by moving whole cells.
template <bool CELL>
__device__ inline void advance_pos(float4& a, float4& d, float h, float ux, float uy, float uz, const Phys& P) {
  if (!CELL) {
    a.x += h * ux;
    a.y += h * uy;
    a.z += h * uz;
    return;
  }
  const uint32_t w = __float_as_uint(d.w);
  int32_t c[3] = {(int32_t)__float_as_uint(d.z), unpack_y(w), unpack_z(w)};
  const float o[3] = {a.x, a.y, a.z}, u[3] = {ux, uy, uz};
  float on[3];
  for (int q = 0; q < 3; ++q) {
    double v = (double)o[q] + (double)h * (double)u[q];
    const double kk = floor(v * P.invS);
    v -= kk * P.S;
    c[q] += (int32_t)kk;
    on[q] = (float)v;
  }
  a.x = on[0];
  a.y = on[1];
  a.z = on[2];
  d.z = __uint_as_float((uint32_t)c[0]);
  d.w = __uint_as_float(pack_yz(c[1], c[2]));
}


__device__ inline void p_taubar(const float s[6], float& p, float& tb) {
  p = -(s[0] + s[1] + s[2]) * (1.0f / 3.0f);
  const float t0 = s[0] + p, t1 = s[1] + p, t2 = s[2] + p;
  tb = fsqrt(0.5f * (t0 * t0 + t1 * t1 + t2 * t2 + 2.f * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5])));
}


}  // namespace crm
