// Reverse-mode (adjoint) kernels of the CRM step for gfx950.
//
// The step (Sec. 2.3: explicit midpoint rule over the rates of Sec. 2.2, BCE of
// Sec. 2.5.1, return mapping of Sec. 2.4) is differentiated with the
// neighbour lists and activity held fixed; at a branch (unilateral viscosity,
// the return-mapping cases, the mu(I) cases) the derivative is the one of the
// branch taken. Each stage is reversed in three passes:
//
//   local   one thread per soil row: adjoint of the row-local parts of the
//           rates (Jaumann term, continuity, dx/dt = u; in stage 2 also the
//           return mapping) and the row's seeds for the pair terms: Lam, the
//           adjoint of its velocity gradient L, and alpha, that of its
//           acceleration;
//   marker  one 8-lane group per marker row: adjoint of the marker's
//           extrapolated velocity and stress (from the seeds of its soil
//           neighbours and, in stage 2, from the seeds of its body's force
//           and torque), then the adjoint of the extrapolation sums;
//   gather  one 8-lane group per soil row: every pair term that involves the
//           row's own state, from its own seeds (the row as i) and from its
//           neighbours' seeds (the row as j). The lists are symmetric, so
//           this is a gather and no scatter or atomic is needed.
//
// Stress vectors are (xx, yy, zz, xy, xz, yz); the adjoint of a stress vector
// has the same layout (derivative with respect to each stored component).
#include "crm_device.h"

namespace crm {
namespace {

// Cubic spline: (dF/dr) / r for F(r) = W'(r) / r, as kg g2(q) with kg = 1 / (pi h^7).
__device__ inline float kernel_g2(float q, float kg) {
  const float t = fmaxf(2.0f - q, 0.0f);
  const float iq = __builtin_amdgcn_rcpf(q);
  const float inner = 2.25f * kg * iq;
  const float outer = 0.75f * kg * (2.0f * t * q + t * t) * iq * iq * iq;
  return q < 1.0f ? inner : outer;
}

// Wendland: (dF/dr) / r = kg t^2 / q, t = 1 - q/2, kg = 15 kw / (2 h^4).
__device__ inline float wendland_g2(float q, float kg) {
  const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
  return kg * t * t * __builtin_amdgcn_rcpf(q);
}

__device__ inline float sph_g2(float q, const Phys& P) {
  return P.kern == 1 ? wendland_g2(q, P.kg) : kernel_g2(q, P.kg);
}

__device__ inline void sym_mv(const float s[6], const float v[3], float o[3]) {
  o[0] = s[0] * v[0] + s[3] * v[1] + s[4] * v[2];
  o[1] = s[3] * v[0] + s[1] * v[1] + s[5] * v[2];
  o[2] = s[4] * v[0] + s[5] * v[1] + s[2] * v[2];
}

// d(a^T S b)/dS for symmetric S in the stored layout, times c.
__device__ inline void sym_outer_add(float g[6], const float a[3], const float b[3], float c) {
  g[0] += c * a[0] * b[0];
  g[1] += c * a[1] * b[1];
  g[2] += c * a[2] * b[2];
  g[3] += c * (a[0] * b[1] + a[1] * b[0]);
  g[4] += c * (a[0] * b[2] + a[2] * b[0]);
  g[5] += c * (a[1] * b[2] + a[2] * b[1]);
}

__device__ inline float dot3(const float a[3], const float b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// H v with H = d(F d)/dd = F I + G2 d d^T.
__device__ inline void hess_mv(float F, float G2, const float d[3], const float v[3], float o[3]) {
  const float t = G2 * dot3(d, v);
  for (int a = 0; a < 3; ++a) o[a] = F * v[a] + t * d[a];
}

// Adjoint of the row-local part of the rates at one evaluation point, from
// the seeds (a_s on ds/dt, a_r on drho/dt) of one row with stress s, density
// rho and velocity gradient L (row-major). Returns the seed Lam on L, the
// direct adjoint of s and rho, and the derivatives with respect to G and K.
struct LocalAdj {
  float lam[9];
  float gs[6];
  float grho;
  float dG, dK;
};

__device__ inline LocalAdj local_adj(const float as[6], float ar, const float s[6], float rho, const float L[9],
                                     const Phys& P) {
  // A = symmetric matrix with A : ds = as . ds (off-diagonals halved)
  const float A[9] = {as[0], 0.5f * as[3], 0.5f * as[4], 0.5f * as[3], as[1], 0.5f * as[5],
                      0.5f * as[4], 0.5f * as[5], as[2]};
  const float S[9] = {s[0], s[3], s[4], s[3], s[1], s[5], s[4], s[5], s[2]};
  float Om[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Om[3 * a + b] = 0.5f * (L[3 * a + b] - L[3 * b + a]);
  const float trA = A[0] + A[4] + A[8];
  const float trL = L[0] + L[4] + L[8];
  LocalAdj o;
  float AD = 0.f;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      float as_ = 0.f, sa = 0.f, ao = 0.f, oa = 0.f;
      for (int k = 0; k < 3; ++k) {
        as_ += A[3 * a + k] * S[3 * k + b];
        sa += S[3 * a + k] * A[3 * k + b];
        ao += A[3 * a + k] * Om[3 * k + b];
        oa += Om[3 * a + k] * A[3 * k + b];
      }
      // d/dL of A : (Om s - s Om) is A s - s A; 2G D and the isotropic term
      o.lam[3 * a + b] = (as_ - sa) + P.two_G * A[3 * a + b] +
                         (a == b ? P.iso * trA - ar * rho : 0.f);
      if (a <= b) {
        // d/ds of A : (Om s - s Om) is A Om - Om A (symmetric)
        const float c = ao - oa;
        if (a == b) o.gs[a] = c;
        else o.gs[a + b + 2] = 2.f * c;   // (0,1)->3, (0,2)->4, (1,2)->5
      }
      AD += A[3 * a + b] * 0.5f * (L[3 * a + b] + L[3 * b + a]);
    }
  o.grho = -ar * trL;
  o.dG = 2.f * AD - (2.f / 3.f) * trL * trA;
  o.dK = P.bulk * trL * trA;
  return o;
}

// Adjoint of the return mapping (Sec. 2.4) for trial stress st, start-of-step
// stress sn and material M = (mu_s, mu_2, cohesion, p_cri), seeded with g on
// the result. Writes the adjoints of st and sn and gp = d/d(mu_s, mu_2,
// cohesion, G). The branch is decided as in the forward mapping.
__device__ inline void return_map_adj(const float st[6], const float sn[6], const Phys& P, float4 M,
                                      const float g[6], float gst[6], float gsn[6], float gp[4]) {
  for (int k = 0; k < 6; ++k) gst[k] = gsn[k] = 0.f;
  gp[0] = gp[1] = gp[2] = gp[3] = 0.f;
  const float mu_s = M.x, mu_2 = M.y, cohesion = M.z;
  float ps, tbs, pn, tbn;
  p_taubar(st, ps, tbs);
  if (ps < M.w) return;                       // tension cut-off: zero stress
  p_taubar(sn, pn, tbn);
  const float gd = (tbs - tbn) * P.inv_Gdt;
  float mu, dmu_s = 0.f, dmu_2 = 0.f, dmu_gd = 0.f, dmu_ps = 0.f;
  if (!(gd > 0.f)) {
    mu = mu_s;
    dmu_s = 1.f;
  } else if (ps <= 0.f) {
    mu = mu_2;
    dmu_2 = 1.f;
  } else {
    const float I = gd * P.grain_d * fsqrt(P.rho0 / ps);
    mu = mu_s + (mu_2 - mu_s) / (1.0f + P.I0 / I);
    const float den = I + P.I0;
    dmu_s = P.I0 / den;
    dmu_2 = I / den;
    const float dmu_I = (mu_2 - mu_s) * P.I0 / (den * den);
    dmu_gd = dmu_I * I / gd;
    dmu_ps = -0.5f * dmu_I * I / ps;
  }
  const float tm = mu * ps + cohesion;
  const bool clamped = !(tm > 0.f);
  const float tmax = clamped ? 0.f : tm;
  if (tbs <= tmax) {                          // admissible trial state
    for (int k = 0; k < 6; ++k) gst[k] = g[k];
    return;
  }
  // radial return: out = -p* I + f tau*, f = tau_max / taubar*
  const float f = tmax / tbs;
  const float tau[6] = {st[0] + ps, st[1] + ps, st[2] + ps, st[3], st[4], st[5]};
  float gf = 0.f;
  for (int k = 0; k < 6; ++k) gf += g[k] * tau[k];
  const float trg = g[0] + g[1] + g[2];
  float g_ps = (f - 1.f) * trg;
  float g_tbs = -gf * f / tbs;
  float g_tbn = 0.f;
  for (int k = 0; k < 6; ++k) gst[k] = f * g[k];
  if (!clamped) {
    const float g_tmax = gf / tbs;
    const float g_mu = g_tmax * ps;
    g_ps += g_tmax * mu + g_mu * dmu_ps;
    gp[0] = g_mu * dmu_s;
    gp[1] = g_mu * dmu_2;
    gp[2] = g_tmax;
    const float g_gd = g_mu * dmu_gd;
    g_tbs += g_gd * P.inv_Gdt;
    g_tbn = -g_gd * P.inv_Gdt;
    gp[3] = -g_gd * gd / P.G;
  }
  for (int k = 0; k < 3; ++k) gst[k] += -g_ps * (1.0f / 3.0f) + g_tbs * tau[k] / (2.f * tbs);
  for (int k = 3; k < 6; ++k) gst[k] += g_tbs * st[k] / tbs;
  if (tbn > 0.f) {
    const float taun[3] = {sn[0] + pn, sn[1] + pn, sn[2] + pn};
    for (int k = 0; k < 3; ++k) gsn[k] = g_tbn * taun[k] / (2.f * tbn);
    for (int k = 3; k < 6; ++k) gsn[k] = g_tbn * sn[k] / tbn;
  }
}

__device__ inline void tape_L(const StageTape& T, int32_t s, float L[9]) {
  const float4 a = T.l0[s], b = T.l1[s], c = T.l2[s];
  L[0] = a.x; L[1] = a.y; L[2] = a.z; L[3] = a.w;
  L[4] = b.x; L[5] = b.y; L[6] = b.z; L[7] = b.w;
  L[8] = c.x;
}

__device__ inline void write_seeds(Planes E, int32_t s, const float lam[9], const float al[3]) {
  E.a[s] = make_float4(lam[0], lam[1], lam[2], lam[3]);
  E.b[s] = make_float4(lam[4], lam[5], lam[6], lam[7]);
  E.c[s] = make_float4(lam[8], al[0], al[1], al[2]);
  E.d[s] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ inline void add_params(float* pg, int32_t s, float dG, float dK, float dms, float dm2, float dc) {
  float* p = pg + (int64_t)s * 5;
  p[0] += dG;
  p[1] += dK;
  p[2] += dms;
  p[3] += dm2;
  p[4] += dc;
}

// Stage 2, row-local part. Ln holds the adjoint of y_{n+1} on entry and the
// adjoint of y_n (identity and return-mapping parts) on exit; Lm gets the
// direct part of the adjoint of y_mid; E the seeds of the pair terms.
__global__ __launch_bounds__(kBlock) void k_adj_local2(const int32_t* __restrict__ rows, int64_t n, Planes Ln,
                                                       Planes Lm, Planes E, CPlanes Yn, CPlanes Ym, StageTape T,
                                                       Phys P, float* __restrict__ pg) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const float4 la = Ln.a[s], lb = Ln.b[s], lc = Ln.c[s], ld = Ln.d[s];
  const float4 t0 = T.t0[s], t1 = T.t1[s];
  const float4 yc = Yn.c[s], yd = Yn.d[s];
  const float st[6] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y};
  const float sn[6] = {yc.x, yc.y, yc.z, yc.w, yd.x, yd.y};
  const float g[6] = {lc.x, lc.y, lc.z, lc.w, ld.x, ld.y};
  float gst[6], gsn[6], gp[4];
  return_map_adj(st, sn, P, P.mat[__float_as_uint(Yn.b[s].w) >> 2], g, gst, gsn, gp);
  // y* = y_n + dt f(y_mid): identity into y_n
  Ln.c[s] = make_float4(gst[0] + gsn[0], gst[1] + gsn[1], gst[2] + gsn[2], gst[3] + gsn[3]);
  Ln.d[s] = make_float4(gst[4] + gsn[4], gst[5] + gsn[5], 0.f, 0.f);
  // seeds of f(y_mid)
  const float h = P.dt;
  const float as[6] = {h * gst[0], h * gst[1], h * gst[2], h * gst[3], h * gst[4], h * gst[5]};
  const float ar = h * la.w;
  const float au[3] = {h * lb.x, h * lb.y, h * lb.z};
  const float ax[3] = {h * la.x, h * la.y, h * la.z};
  const float4 mc = Ym.c[s], md = Ym.d[s];
  const float sm[6] = {mc.x, mc.y, mc.z, mc.w, md.x, md.y};
  float L[9];
  tape_L(T, s, L);
  const LocalAdj o = local_adj(as, ar, sm, Ym.a[s].w, L, P);
  Lm.a[s] = make_float4(0.f, 0.f, 0.f, o.grho);
  Lm.b[s] = make_float4(ax[0], ax[1], ax[2], 0.f);
  Lm.c[s] = make_float4(o.gs[0], o.gs[1], o.gs[2], o.gs[3]);
  Lm.d[s] = make_float4(o.gs[4], o.gs[5], 0.f, 0.f);
  write_seeds(E, s, o.lam, au);
  add_params(pg, s, o.dG + gp[3], o.dK, gp[0], gp[1], gp[2]);
}

// Stage 1, row-local part: y_mid = y_n + dt/2 f(y_n). Ln += Lm + the direct
// part at y_n; E gets the seeds.
__global__ __launch_bounds__(kBlock) void k_adj_local1(const int32_t* __restrict__ rows, int64_t n, Planes Ln,
                                                       CPlanes Lm, Planes E, CPlanes Yn, StageTape T, Phys P,
                                                       float* __restrict__ pg) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const float4 ma = Lm.a[s], mb = Lm.b[s], mc = Lm.c[s], md = Lm.d[s];
  const float h = P.half_dt;
  const float as[6] = {h * mc.x, h * mc.y, h * mc.z, h * mc.w, h * md.x, h * md.y};
  const float ar = h * ma.w;
  const float au[3] = {h * mb.x, h * mb.y, h * mb.z};
  const float ax[3] = {h * ma.x, h * ma.y, h * ma.z};
  const float4 yc = Yn.c[s], yd = Yn.d[s];
  const float sn[6] = {yc.x, yc.y, yc.z, yc.w, yd.x, yd.y};
  float L[9];
  tape_L(T, s, L);
  const LocalAdj o = local_adj(as, ar, sn, Yn.a[s].w, L, P);
  const float4 na = Ln.a[s], nb = Ln.b[s], nc = Ln.c[s], nd = Ln.d[s];
  Ln.a[s] = make_float4(na.x + ma.x, na.y + ma.y, na.z + ma.z, na.w + ma.w + o.grho);
  Ln.b[s] = make_float4(nb.x + mb.x + ax[0], nb.y + mb.y + ax[1], nb.z + mb.z + ax[2], 0.f);
  Ln.c[s] = make_float4(nc.x + mc.x + o.gs[0], nc.y + mc.y + o.gs[1], nc.z + mc.z + o.gs[2], nc.w + mc.w + o.gs[3]);
  Ln.d[s] = make_float4(nd.x + md.x + o.gs[4], nd.y + md.y + o.gs[5], 0.f, 0.f);
  write_seeds(E, s, o.lam, au);
  add_params(pg, s, o.dG, o.dK, 0.f, 0.f, 0.f);
}

__device__ inline void load_state(const Nbr& o, float u[3], float sg[6]) {
  u[0] = o.b.x; u[1] = o.b.y; u[2] = o.b.z;
  sg[0] = o.c.x; sg[1] = o.c.y; sg[2] = o.c.z; sg[3] = o.c.w; sg[4] = o.d.x; sg[5] = o.d.y;
}

// Marker rows. With FORCE (stage 2) the marker's acceleration enters its
// body's force and torque, seeded by fs = (lambda_F, lambda_T) per body:
// beta = m (lambda_F + lambda_T x r). The adjoint of the marker's extrapolated
// velocity and stress is gathered from the seeds of its soil neighbours and
// from beta; the adjoints of the extrapolation sums go to E:
//   a = (l_su, l_Z)  b = l_ss[0..3]  c = (l_ss[4..5], l_sr[0..1])  d = (l_sr[2], beta)
template <bool FORCE, bool CELL>
__global__ __launch_bounds__(kBlock) void k_adj_marker(CPlanes Y, Planes E, const int32_t* __restrict__ mrows,
                                                       int64_t n, const uint64_t* __restrict__ off,
                                                       const uint32_t* __restrict__ nbr,
                                                       const Body* __restrict__ bodies, const double* __restrict__ fs,
                                                       Phys P, float* __restrict__ pg) {
  const int64_t r = (xcd_block() * kBlock + threadIdx.x) / kGroup;
  const int gl = group_lane();
  const bool live = r < n;
  int32_t s = 0;
  int body = 0;
  float4 ma = make_float4(0.f, 0.f, 0.f, 1.f), mb = make_float4(0.f, 0.f, 0.f, 0.f), mc = mb, md = mb;
  uint64_t k0 = 0, k1 = 0;
  if (live) {
    s = mrows[r];
    ma = Y.a[s]; mb = Y.b[s]; mc = Y.c[s]; md = Y.d[s];
    body = (int)(__float_as_uint(mb.w) >> 2);
    k0 = off[r];
    k1 = off[r + 1];
  }
  const Own me = own_pos<CELL>(ma, md);
  const float rhos = ma.w;
  const float us[3] = {mb.x, mb.y, mb.z};
  const float ss_[6] = {mc.x, mc.y, mc.z, mc.w, md.x, md.y};
  // lever arm, body acceleration at the marker and the force seed
  double rv[3] = {0.0, 0.0, 0.0};
  float asb[3] = {0.f, 0.f, 0.f}, beta[3] = {0.f, 0.f, 0.f};
  if (live) {
    const Body& Bd = bodies[body];
    if (CELL) {
      rv[0] = from_cell(me.cx, me.x, P.lo[0], P.S) - Bd.X[0];
      rv[1] = from_cell(me.cy, me.y, P.lo[1], P.S) - Bd.X[1];
      rv[2] = from_cell(me.cz, me.z, P.lo[2], P.S) - Bd.X[2];
    } else {
      rv[0] = (double)me.x - Bd.X[0];
      rv[1] = (double)me.y - Bd.X[1];
      rv[2] = (double)me.z - Bd.X[2];
    }
    const double wr[3] = {Bd.W[1] * rv[2] - Bd.W[2] * rv[1], Bd.W[2] * rv[0] - Bd.W[0] * rv[2],
                          Bd.W[0] * rv[1] - Bd.W[1] * rv[0]};
    const double wwr[3] = {Bd.W[1] * wr[2] - Bd.W[2] * wr[1], Bd.W[2] * wr[0] - Bd.W[0] * wr[2],
                           Bd.W[0] * wr[1] - Bd.W[1] * wr[0]};
    if (Bd.has_acc) {
      const double ar[3] = {Bd.Al[1] * rv[2] - Bd.Al[2] * rv[1], Bd.Al[2] * rv[0] - Bd.Al[0] * rv[2],
                            Bd.Al[0] * rv[1] - Bd.Al[1] * rv[0]};
      for (int a = 0; a < 3; ++a) asb[a] = (float)(Bd.A[a] + ar[a] + wwr[a]);
    } else {
      for (int a = 0; a < 3; ++a) asb[a] = (float)wwr[a];
    }
    if (FORCE) {
      const double* f = fs + 6 * body;
      const double tr[3] = {f[4] * rv[2] - f[5] * rv[1], f[5] * rv[0] - f[3] * rv[2], f[3] * rv[1] - f[4] * rv[0]};
      for (int a = 0; a < 3; ++a) beta[a] = (float)((double)P.m * (f[a] + tr[a]));
    }
  }
  const float Vs = P.m / rhos;
  float sw = 0.f, su[3] = {0.f, 0.f, 0.f}, sS[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, sr[3] = {0.f, 0.f, 0.f};
  float lu[3] = {0.f, 0.f, 0.f}, ls[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, gK = 0.f;
  walk_row(Y, k0, k1, nbr, [&](const Nbr& o, uint32_t j) {
    float d[3];
    pair_sep<CELL>(me, o, P.Sf, d[0], d[1], d[2]);
    const float r2 = dot3(d, d);
    const float q = fsqrt(r2) * P.inv_h;
    const float F = sph_f(q, P);
    const float W = sph_w(q, P);
    float uf[3], sf[6];
    load_state(o, uf, sf);
    const float rhof = o.a.w;
    sw += W;
    for (int a = 0; a < 3; ++a) su[a] += uf[a] * W;
    for (int a = 0; a < 6; ++a) sS[a] += sf[a] * W;
    for (int a = 0; a < 3; ++a) sr[a] += rhof * W * d[a];
    const float v[3] = {us[0] - uf[0], us[1] - uf[1], us[2] - uf[2]};
    const float vr = dot3(v, d);
    const bool av = P.av_mode == 1 || (P.av_mode == 2 && vr < 0.f);
    const float Q = av ? P.av_coef * F * __builtin_amdgcn_rcpf(0.5f * (rhos + rhof) * (r2 + P.xi2)) : 0.f;
    if ((__float_as_uint(o.b.w) & 3u) == kSoilActive) {
      // soil row j with this marker as neighbour
      const float4 ea = at(E.a, j), eb = at(E.b, j), ec = at(E.c, j);
      const float lam[9] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w, ec.x};
      const float al[3] = {ec.y, ec.z, ec.w};
      const float ad = dot3(al, d);
      for (int a = 0; a < 3; ++a) {
        const float ld = lam[3 * a] * d[0] + lam[3 * a + 1] * d[1] + lam[3 * a + 2] * d[2];
        lu[a] += -Vs * F * ld - Q * ad * d[a];
      }
      sym_outer_add(ls, al, d, -Vs * F / rhof);
    }
    if (FORCE) {
      const float bd = dot3(beta, d);
      sym_outer_add(ls, beta, d, P.m / rhof * F / rhos);
      for (int a = 0; a < 3; ++a) lu[a] += Q * bd * d[a];
      gK += Q * vr * bd * P.inv_2K;
    }
  });
  sw = group_sum(sw);
  for (int a = 0; a < 3; ++a) {
    su[a] = group_sum(su[a]);
    sr[a] = group_sum(sr[a]);
    lu[a] = group_sum(lu[a]);
  }
  for (int a = 0; a < 6; ++a) {
    sS[a] = group_sum(sS[a]);
    ls[a] = group_sum(ls[a]);
  }
  gK = group_sum(gK);
  (void)ss_;
  if (!live) return;
  float lsu[3] = {0.f, 0.f, 0.f}, lss[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, lsr[3] = {0.f, 0.f, 0.f}, lZ = 0.f;
  if (sw > 0.f) {
    const float iw = 1.0f / sw;
    const float gdv = ((P.gx - asb[0]) * sr[0] + (P.gy - asb[1]) * sr[1]) + (P.gz - asb[2]) * sr[2];
    const float sg[6] = {(sS[0] - gdv) * iw, (sS[1] - gdv) * iw, (sS[2] - gdv) * iw, sS[3] * iw, sS[4] * iw,
                         sS[5] * iw};
    for (int a = 0; a < 3; ++a) lsu[a] = -lu[a] * iw;
    for (int a = 0; a < 6; ++a) lss[a] = ls[a] * iw;
    const float lgd = -(ls[0] + ls[1] + ls[2]) * iw;
    lsr[0] = lgd * (P.gx - asb[0]);
    lsr[1] = lgd * (P.gy - asb[1]);
    lsr[2] = lgd * (P.gz - asb[2]);
    float sdot = 0.f;
    for (int a = 0; a < 6; ++a) sdot += ls[a] * sg[a];
    lZ = dot3(lu, su) * iw * iw - sdot * iw;
  }
  float4 v;
  float4* dst;
  if (gl == 0) { v = make_float4(lsu[0], lsu[1], lsu[2], lZ); dst = E.a; }
  else if (gl == 1) { v = make_float4(lss[0], lss[1], lss[2], lss[3]); dst = E.b; }
  else if (gl == 2) { v = make_float4(lss[4], lss[5], lsr[0], lsr[1]); dst = E.c; }
  else { v = make_float4(lsr[2], beta[0], beta[1], beta[2]); dst = E.d; }
  if (gl < 4) dst[s] = v;
  if (FORCE && gl == 4 % kGroup) pg[(int64_t)s * 5 + 1] += gK;
}

// Soil rows: all pair terms that involve the row's own state, added to the
// adjoint planes Lt (the adjoint of the stage's evaluation point).
template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_adj_gather(CPlanes Y, CPlanes E, const int32_t* __restrict__ rows,
                                                       int64_t n, const uint64_t* __restrict__ off,
                                                       const uint32_t* __restrict__ nbr, Phys P, Planes Lt,
                                                       float* __restrict__ pg) {
  const int64_t r = (xcd_block() * kBlock + threadIdx.x) / kGroup;
  const int gl = group_lane();
  const bool live = r < n;
  int32_t s = 0;
  float4 ma = make_float4(0.f, 0.f, 0.f, 1.f), mb = make_float4(0.f, 0.f, 0.f, 0.f), mc = mb, md = mb;
  float4 ea = mb, eb = mb, ec = mb;
  uint64_t k0 = 0, k1 = 0;
  if (live) {
    s = rows[r];
    ma = Y.a[s]; mb = Y.b[s]; mc = Y.c[s]; md = Y.d[s];
    ea = E.a[s]; eb = E.b[s]; ec = E.c[s];
    k0 = off[r];
    k1 = off[r + 1];
  }
  const Own me = own_pos<CELL>(ma, md);
  const float rhop = ma.w;
  const float up[3] = {mb.x, mb.y, mb.z};
  const float sp[6] = {mc.x, mc.y, mc.z, mc.w, md.x, md.y};
  const float lam[9] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w, ec.x};
  const float al[3] = {ec.y, ec.z, ec.w};
  const float Vp = P.m / rhop;
  float gx[3] = {0.f, 0.f, 0.f}, gu[3] = {0.f, 0.f, 0.f}, gs[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gr = 0.f, gK = 0.f;
  walk_row(Y, k0, k1, nbr, [&](const Nbr& o, uint32_t j) {
    if (j == (uint32_t)s) return;                       // self pair: no term
    float d[3];
    pair_sep<CELL>(me, o, P.Sf, d[0], d[1], d[2]);
    const float r2 = dot3(d, d);
    if (!(r2 > 0.f)) return;
    const float q = fsqrt(r2) * P.inv_h;
    const float F = sph_f(q, P);
    const float G2 = sph_g2(q, P);
    float uq[3], sq[6];
    load_state(o, uq, sq);
    const float rhoq = o.a.w;
    const uint32_t kind = __float_as_uint(o.b.w) & 3u;
    const float Vq = P.m / rhoq;
    const float du[3] = {uq[0] - up[0], uq[1] - up[1], uq[2] - up[2]};   // u_j - u_i
    const float v[3] = {-du[0], -du[1], -du[2]};                         // u_i - u_j
    const float vr = dot3(v, d);
    const float S[6] = {sp[0] + sq[0], sp[1] + sq[1], sp[2] + sq[2], sp[3] + sq[3], sp[4] + sq[4], sp[5] + sq[5]};
    const bool av = P.av_mode == 1 || (P.av_mode == 2 && vr < 0.f);
    const float rbar = 0.5f * (rhop + rhoq);
    const float D2 = r2 + P.xi2;
    const float iD2 = __builtin_amdgcn_rcpf(D2);
    const float cv = av ? P.av_coef * __builtin_amdgcn_rcpf(rbar) : 0.f;
    const float Q = cv * F * iD2;
    float h[3], t[3];
    // ---- the row as i: its own seeds (lam, al)
    {
      float ld[3], lt[3], sa[3];
      for (int a = 0; a < 3; ++a) {
        ld[a] = lam[3 * a] * d[0] + lam[3 * a + 1] * d[1] + lam[3 * a + 2] * d[2];
        lt[a] = lam[a] * du[0] + lam[3 + a] * du[1] + lam[6 + a] * du[2];
      }
      sym_mv(S, al, sa);
      const float ad = dot3(al, d);
      const float phiA = Vq * F / rhop * dot3(sa, d);
      const float phiV = Q * vr * ad;
      for (int a = 0; a < 3; ++a) gu[a] += -Vq * F * ld[a] + Q * ad * d[a];
      sym_outer_add(gs, al, d, Vq * F / rhop);
      gr += -phiA / rhop - 0.5f * phiV / rbar;
      hess_mv(F, G2, d, lt, h);
      for (int a = 0; a < 3; ++a) gx[a] += Vq * h[a];
      hess_mv(F, G2, d, sa, h);
      for (int a = 0; a < 3; ++a) gx[a] += Vq / rhop * h[a];
      if (av) {
        const float ag = F * ad;
        hess_mv(F, G2, d, al, h);
        for (int a = 0; a < 3; ++a) gx[a] += cv * (ag * iD2 * v[a] + vr * iD2 * h[a] - 2.f * vr * ag * iD2 * iD2 * d[a]);
      }
      gK += phiV * P.inv_2K;
    }
    // ---- the row as j of its neighbour's terms
    const bool is_marker = kind == kMarker;
    if (kind == kSoilActive || is_marker) {
      const float4 fa = at(E.a, j), fb = at(E.b, j), fc = at(E.c, j), fd = at(E.d, j);
      float lq[9], aq[3];
      if (is_marker) {
        for (int a = 0; a < 9; ++a) lq[a] = 0.f;
        aq[0] = fd.y; aq[1] = fd.z; aq[2] = fd.w;      // beta of the marker's force
      } else {
        lq[0] = fa.x; lq[1] = fa.y; lq[2] = fa.z; lq[3] = fa.w;
        lq[4] = fb.x; lq[5] = fb.y; lq[6] = fb.z; lq[7] = fb.w; lq[8] = fc.x;
        aq[0] = fc.y; aq[1] = fc.z; aq[2] = fc.w;
      }
      float ld[3], lt[3], sa[3];
      for (int a = 0; a < 3; ++a) {
        ld[a] = lq[3 * a] * d[0] + lq[3 * a + 1] * d[1] + lq[3 * a + 2] * d[2];
        lt[a] = lq[a] * v[0] + lq[3 + a] * v[1] + lq[6 + a] * v[2];
      }
      sym_mv(S, aq, sa);
      const float ad = dot3(aq, d);
      const float phiL = -Vp * F * dot3(v, ld);
      const float phiA = -Vp * F / rhoq * dot3(sa, d);
      const float phiV = -Q * vr * ad;
      for (int a = 0; a < 3; ++a) gu[a] += -Vp * F * ld[a] - Q * ad * d[a];
      sym_outer_add(gs, aq, d, -Vp * F / rhoq);
      gr += -(phiL + phiA) / rhop - 0.5f * phiV / rbar;
      hess_mv(F, G2, d, lt, h);
      for (int a = 0; a < 3; ++a) gx[a] -= Vp * h[a];
      hess_mv(F, G2, d, sa, h);
      for (int a = 0; a < 3; ++a) gx[a] -= Vp / rhoq * h[a];
      if (av) {
        const float ag = F * ad;
        hess_mv(F, G2, d, aq, t);
        for (int a = 0; a < 3; ++a) gx[a] -= cv * (ag * iD2 * v[a] + vr * iD2 * t[a] - 2.f * vr * ag * iD2 * iD2 * d[a]);
      }
      if (is_marker) {
        // the marker's extrapolation sums over this soil particle (Sec. 2.5.1)
        const float W = sph_w(q, P);
        const float lsu[3] = {fa.x, fa.y, fa.z};
        const float lss[6] = {fb.x, fb.y, fb.z, fb.w, fc.x, fc.y};
        const float lsr[3] = {fc.z, fc.w, fd.x};
        const float lsd = dot3(lsr, d);
        float ssd = 0.f;
        for (int a = 0; a < 6; ++a) {
          gs[a] += lss[a] * W;
          ssd += lss[a] * sp[a];
        }
        for (int a = 0; a < 3; ++a) gu[a] += lsu[a] * W;
        gr += -lsd * W;
        const float coef = dot3(lsu, up) + ssd - rhop * lsd + fa.w;
        for (int a = 0; a < 3; ++a) gx[a] += coef * F * d[a] - rhop * W * lsr[a];
      }
    }
  });
  for (int a = 0; a < 3; ++a) {
    gx[a] = group_sum(gx[a]);
    gu[a] = group_sum(gu[a]);
  }
  for (int a = 0; a < 6; ++a) gs[a] = group_sum(gs[a]);
  gr = group_sum(gr);
  gK = group_sum(gK);
  if (!live) return;
  // lanes 0-3 each update one plane of the row's adjoint record
  float4* dst = gl == 0 ? Lt.a : gl == 1 ? Lt.b : gl == 2 ? Lt.c : Lt.d;
  if (gl < 4) {
    float4 w = dst[s];
    if (gl == 0) { w.x += gx[0]; w.y += gx[1]; w.z += gx[2]; w.w += gr; }
    else if (gl == 1) { w.x += gu[0]; w.y += gu[1]; w.z += gu[2]; }
    else if (gl == 2) { w.x += gs[0]; w.y += gs[1]; w.z += gs[2]; w.w += gs[3]; }
    else { w.x += gs[4]; w.y += gs[5]; }
    dst[s] = w;
  }
  if (gl == 4 % kGroup) pg[(int64_t)s * 5 + 1] += gK;
}

// Adjoint records between particle-id order and slot order.
__global__ __launch_bounds__(kBlock) void k_adj_to_slots(const int32_t* __restrict__ rows, int64_t n,
                                                         const int32_t* __restrict__ slot_id, CPlanes byid,
                                                         Planes byslot) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const int32_t i = slot_id[s];
  byslot.a[s] = byid.a[i];
  byslot.b[s] = byid.b[i];
  byslot.c[s] = byid.c[i];
  byslot.d[s] = byid.d[i];
}

__global__ __launch_bounds__(kBlock) void k_adj_to_ids(const int32_t* __restrict__ rows, int64_t n,
                                                       const int32_t* __restrict__ slot_id, CPlanes byslot,
                                                       Planes byid) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t s = rows[r];
  const int32_t i = slot_id[s];
  byid.a[i] = byslot.a[s];
  byid.b[i] = byslot.b[s];
  byid.c[i] = byslot.c[s];
  byid.d[i] = byslot.d[s];
}

// Per-slot parameter partials (FP32, one segment of steps) into per-id FP64
// accumulators; every slot of the processed set maps to one id.
__global__ __launch_bounds__(kBlock) void k_adj_params_to_ids(int64_t n_proc, const int32_t* __restrict__ slot_id,
                                                              float* __restrict__ pg, double* __restrict__ pid) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= n_proc) return;
  const int64_t i = slot_id[s];
  for (int k = 0; k < 5; ++k) {
    pid[i * 6 + k] += (double)pg[s * 5 + k];
    pg[s * 5 + k] = 0.f;
  }
}

// Per-id accumulators in group order (perm) for the fixed-order group sums.
__global__ __launch_bounds__(kBlock) void k_adj_params_permute(int64_t n, const int32_t* __restrict__ perm,
                                                               const double* __restrict__ pid,
                                                               double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int64_t i = perm[k];
  for (int a = 0; a < 6; ++a) out[k * 6 + a] = pid[i * 6 + a];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned nblk_groups(int64_t rows) { return nblk(rows * kGroup); }

// Seeds of the end state, from the caller's flat arrays (any may be absent)
// into the adjoint planes by particle id: a = (x, y, z, rho), b = (u, -),
// c, d = stress.
__global__ __launch_bounds__(kBlock) void k_adj_pack(int64_t n, const double* __restrict__ pos,
                                                     const float* __restrict__ vel, const float* __restrict__ sig,
                                                     const float* __restrict__ rho, Planes out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a, d = a;
  if (pos) a = make_float4((float)pos[3 * i], (float)pos[3 * i + 1], (float)pos[3 * i + 2], 0.f);
  if (rho) a.w = rho[i];
  if (vel) b = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
  if (sig) {
    c = make_float4(sig[6 * i], sig[6 * i + 1], sig[6 * i + 2], sig[6 * i + 3]);
    d = make_float4(sig[6 * i + 4], sig[6 * i + 5], 0.f, 0.f);
  }
  out.a[i] = a;
  out.b[i] = b;
  out.c[i] = c;
  out.d[i] = d;
}

// The adjoint of the start state into flat arrays (any may be absent); bad
// is set when any of the 13 values of a particle is not finite.
__global__ __launch_bounds__(kBlock) void k_adj_unpack(int64_t n, CPlanes in, double* __restrict__ pos,
                                                       float* __restrict__ vel, float* __restrict__ sig,
                                                       float* __restrict__ rho, uint32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 a = in.a[i], b = in.b[i], c = in.c[i], d = in.d[i];
  const float v[13] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, c.x, c.y, c.z, c.w, d.x, d.y};
  bool fin = true;
  for (float x : v) fin = fin && isfinite(x);
  if (!fin) atomicOr(bad, 1u);
  if (pos) {
    pos[3 * i] = a.x;
    pos[3 * i + 1] = a.y;
    pos[3 * i + 2] = a.z;
  }
  if (rho) rho[i] = a.w;
  if (vel) {
    vel[3 * i] = b.x;
    vel[3 * i + 1] = b.y;
    vel[3 * i + 2] = b.z;
  }
  if (sig) {
    sig[6 * i] = c.x;
    sig[6 * i + 1] = c.y;
    sig[6 * i + 2] = c.z;
    sig[6 * i + 3] = c.w;
    sig[6 * i + 4] = d.x;
    sig[6 * i + 5] = d.y;
  }
}

}  // namespace

hipError_t adj_local2(const int32_t* rows, int64_t n, Planes Ln, Planes Lm, Planes E, CPlanes Yn, CPlanes Ym,
                      const StageTape& T, Phys P, float* pg, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_local2<<<nblk(n), kBlock, 0, s>>>(rows, n, Ln, Lm, E, Yn, Ym, T, P, pg);
  return hipGetLastError();
}

hipError_t adj_local1(const int32_t* rows, int64_t n, Planes Ln, CPlanes Lm, Planes E, CPlanes Yn,
                      const StageTape& T, Phys P, float* pg, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_local1<<<nblk(n), kBlock, 0, s>>>(rows, n, Ln, Lm, E, Yn, T, P, pg);
  return hipGetLastError();
}

hipError_t adj_marker(CPlanes Y, Planes E, const int32_t* mrows, int64_t n, const uint64_t* off,
                      const uint32_t* nbr, const Body* bodies, const double* fs, Phys P, float* pg,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = nblk_groups(n);
  if (P.cell) {
    if (fs) k_adj_marker<true, true><<<g, kBlock, 0, s>>>(Y, E, mrows, n, off, nbr, bodies, fs, P, pg);
    else k_adj_marker<false, true><<<g, kBlock, 0, s>>>(Y, E, mrows, n, off, nbr, bodies, fs, P, pg);
  } else {
    if (fs) k_adj_marker<true, false><<<g, kBlock, 0, s>>>(Y, E, mrows, n, off, nbr, bodies, fs, P, pg);
    else k_adj_marker<false, false><<<g, kBlock, 0, s>>>(Y, E, mrows, n, off, nbr, bodies, fs, P, pg);
  }
  return hipGetLastError();
}

hipError_t adj_gather(CPlanes Y, CPlanes E, const int32_t* rows, int64_t n, const uint64_t* off,
                      const uint32_t* nbr, Phys P, Planes Lt, float* pg, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = nblk_groups(n);
  if (P.cell) k_adj_gather<true><<<g, kBlock, 0, s>>>(Y, E, rows, n, off, nbr, P, Lt, pg);
  else k_adj_gather<false><<<g, kBlock, 0, s>>>(Y, E, rows, n, off, nbr, P, Lt, pg);
  return hipGetLastError();
}

hipError_t adj_to_slots(const int32_t* rows, int64_t n, const int32_t* slot_id, CPlanes byid, Planes byslot,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_to_slots<<<nblk(n), kBlock, 0, s>>>(rows, n, slot_id, byid, byslot);
  return hipGetLastError();
}

hipError_t adj_to_ids(const int32_t* rows, int64_t n, const int32_t* slot_id, CPlanes byslot, Planes byid,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_to_ids<<<nblk(n), kBlock, 0, s>>>(rows, n, slot_id, byslot, byid);
  return hipGetLastError();
}

hipError_t adj_params_to_ids(int64_t n_proc, const int32_t* slot_id, float* pg, double* pid, hipStream_t s) {
  if (n_proc <= 0) return hipSuccess;
  k_adj_params_to_ids<<<nblk(n_proc), kBlock, 0, s>>>(n_proc, slot_id, pg, pid);
  return hipGetLastError();
}

hipError_t adj_pack(int64_t n, const double* pos, const float* vel, const float* sig, const float* rho, Planes out,
                    hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_pack<<<nblk(n), kBlock, 0, s>>>(n, pos, vel, sig, rho, out);
  return hipGetLastError();
}

hipError_t adj_unpack(int64_t n, CPlanes in, double* pos, float* vel, float* sig, float* rho, uint32_t* bad,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_unpack<<<nblk(n), kBlock, 0, s>>>(n, in, pos, vel, sig, rho, bad);
  return hipGetLastError();
}

hipError_t adj_params_permute(int64_t n, const int32_t* perm, const double* pid, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adj_params_permute<<<nblk(n), kBlock, 0, s>>>(n, perm, pid, out);
  return hipGetLastError();
}

}  // namespace crm
