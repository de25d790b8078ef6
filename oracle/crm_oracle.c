/*
 * crm_oracle.c -- FP64 CPU oracle of the CRM particle step.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file; the product library never does. It
 * shares no code with the HIP path.
 *
 * What it computes, in the paper's order (arXiv 2507.05643):
 *   - cubic spline kernel W with support 2h (Sec. 4.1, kernel list; Monaghan 1985)
 *   - neighbour sets {j : |x_i - x_j| < 2h} by brute force (the definition), and
 *     by the cell-linked list of Sec. 4.1 steps 1-4 (hash c = z*Y*X + y*X + x,
 *     sort by cell, cellStart/cellEnd, 27-cell scan of Algorithm 1)
 *   - persistent lists rebuilt when step mod ps_freq == 0 (Algorithm 2)
 *   - active domains: Active / Extended-Active / Inactive flags from oriented
 *     boxes attached to bodies, compaction, capacity policy (Sec. 4.2, Alg. 3)
 *   - BCE markers: Adami velocity extrapolation with no-slip correction and
 *     stress extrapolation (Sec. 2.5.1)
 *   - discrete continuity (F2), momentum (F3) with artificial viscosity, and
 *     Jaumann hypo-elastic stress rate (Sec. 2.2, eqs. continuity_dis,
 *     momentum_dis, stress_rate_dis, artificial_viscosity_*)
 *   - explicit midpoint RK2 (Sec. 2.3)
 *   - four-step cohesive mu(I) return mapping after the full step (Sec. 2.4)
 *   - body force and torque from marker accelerations (Sec. 2.5.1)
 *
 * Readings where the paper is silent or garbled are listed in the design notes
 * of the repository and referenced here by their subject.
 *
 * Plain loops, FP64, one particle at a time; the only library routine used is
 * qsort (for the sort-by-cell step).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct orc_params {
  double dx, h, dt;
  double g[3];
  double rho0, E, nu, mu_s, mu_2, I0, grain_d, cohesion;
  double av_gamma, av_xi_over_h;
  int32_t av_mode;        /* 0 off, 1 bilateral, 2 unilateral */
  int32_t ps_freq;
  double lo[3], hi[3];
  int32_t periodic[3];    /* oracle-only: minimum-image distances on these axes */
  int32_t active_domains;
  double t_delay;
  double grow_G, shrink_S;
  int32_t shrink_interval;
  int32_t nbr_mode;       /* 0 brute force, 1 cell list */
  double bulk_coeff;      /* factor on the bulk term K tr(D) I (1 = continuum form) */
  int32_t pos_mode;       /* stored position form of the kernel: 0 FP32 absolute,
                             1 cell index + FP32 offset */
  int32_t kernel;         /* smoothing kernel: 0 cubic spline, 1 quintic Wendland */
} orc_params;

/* ------------------------------------------------------------------ kernel */
/* Cubic spline (Monaghan 1985), q = r/h, support q < 2, 3-D normalisation
 * 1/(pi h^3). The paper names the kernel and its support 2h (Sec. 4.1). */
double orc_W(double r, double h) {
  double q = r / h, s = 1.0 / (ORC_PI * h * h * h);
  if (q < 1.0) return s * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
  if (q < 2.0) { double t = 2.0 - q; return s * 0.25 * t * t * t; }
  return 0.0;
}

/* dW/dr of the same kernel. */
double orc_dWdr(double r, double h) {
  double q = r / h, s = 1.0 / (ORC_PI * h * h * h * h);
  if (q < 1.0) return s * (-3.0 * q + 2.25 * q * q);
  if (q < 2.0) { double t = 2.0 - q; return s * (-0.75 * t * t); }
  return 0.0;
}

/* Quintic Wendland C2 kernel (Wendland 1995; the alternative the paper's
 * solver offers, Sec. 4.1), support q < 2, 3-D normalisation 21/(16 pi h^3):
 * W = a (1 - q/2)^4 (2q + 1). */
double orc_W_wendland(double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double a = 21.0 / (16.0 * ORC_PI * h * h * h), t = 1.0 - 0.5 * q;
  return a * t * t * t * t * (2.0 * q + 1.0);
}

/* dW/dr of the Wendland kernel: -5 a q (1 - q/2)^3 / h. */
double orc_dWdr_wendland(double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double a = 21.0 / (16.0 * ORC_PI * h * h * h), t = 1.0 - 0.5 * q;
  return -5.0 * a * q * t * t * t / h;
}

static double kern_W(const orc_params* P, double r) {
  return P->kernel == 1 ? orc_W_wendland(r, P->h) : orc_W(r, P->h);
}

static double kern_dWdr(const orc_params* P, double r) {
  return P->kernel == 1 ? orc_dWdr_wendland(r, P->h) : orc_dWdr(r, P->h);
}

/* grad_i W_ij = dW/dr * (x_i - x_j) / r; zero for r = 0 (the self pair). */
static void gradW(const orc_params* P, const double rij[3], double r, double out[3]) {
  if (r <= 0.0) { out[0] = out[1] = out[2] = 0.0; return; }
  double f = kern_dWdr(P, r) / r;
  out[0] = f * rij[0]; out[1] = f * rij[1]; out[2] = f * rij[2];
}

/* Separation x_i - x_j, with minimum image on periodic axes (oracle only). */
static void sep(const orc_params* P, const double* xi, const double* xj, double out[3]) {
  for (int a = 0; a < 3; ++a) {
    double d = xi[a] - xj[a];
    if (P->periodic[a]) {
      double L = P->hi[a] - P->lo[a];
      if (d > 0.5 * L) d -= L;
      else if (d < -0.5 * L) d += L;
    }
    out[a] = d;
  }
}

/* ------------------------------------------------------- neighbour search */
/* Integer decisions (cell of a particle, neighbour membership, activity) are
 * taken on the position as the kernel stores it, so both sides decide the
 * same way. pos_mode 0: FP32 absolute coordinates. pos_mode 1: integer cell
 * coordinate c = floor((x - lo) / (2h)) and FP32 offset o = x - lo - c 2h (the
 * physics of the oracle stays FP64 in both modes). */
typedef struct { int64_t c[3]; double o[3]; } rep_t;

static void to_rep(const orc_params* P, const double* x, rep_t* r) {
  const double S = 2.0 * P->h, inv = 1.0 / S;
  for (int a = 0; a < 3; ++a) {
    if (P->pos_mode == 1) {
      double t = x[a] - P->lo[a];
      double c = floor(t * inv);
      r->c[a] = (int64_t)c;
      r->o[a] = (double)(float)(t - c * S);
    } else {
      r->c[a] = 0;
      r->o[a] = (double)(float)x[a];
    }
  }
}

/* Absolute FP64 position of a stored representation. */
static void rep_abs(const orc_params* P, const rep_t* r, double* x) {
  const double S = 2.0 * P->h;
  for (int a = 0; a < 3; ++a)
    x[a] = (P->pos_mode == 1) ? (P->lo[a] + (double)r->c[a] * S) + r->o[a] : r->o[a];
}

/* Neighbour predicate: |x_i - x_j| < 2h in FP64 on the stored positions, as
 * ((dx^2 + dy^2) + dz^2) < (2h)^2 with dx = (c_i - c_j) 2h + (o_i - o_j). The
 * self pair is included (Algorithm 1 scans the particle's own cell). */
static int is_nbr(const orc_params* P, const double* xi, const double* xj) {
  rep_t a, b;
  to_rep(P, xi, &a);
  to_rep(P, xj, &b);
  const double S = 2.0 * P->h;
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = (double)(a.c[k] - b.c[k]) * S + (a.o[k] - b.o[k]);
  if (P->pos_mode == 0) {
    double aa[3] = {a.o[0], a.o[1], a.o[2]}, bb[3] = {b.o[0], b.o[1], b.o[2]};
    sep(P, aa, bb, d);
  }
  double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
  double R = 2.0 * P->h;
  return r2 < R * R;
}

/* Brute force over all pairs of the set `ids` (ascending ids). Lists are in
 * CSR form indexed by position in `ids`; neighbour entries are particle ids in
 * ascending order. Returns the number of entries, or -1 if cap is exceeded. */
int64_t orc_neighbors_brute(const orc_params* P, int64_t n_set, const int32_t* ids,
                            const double* x, int64_t* off, int32_t* nbr, int64_t cap) {
  int64_t tot = 0;
  for (int64_t a = 0; a < n_set; ++a) {
    off[a] = tot;
    const double* xi = x + 3 * (int64_t)ids[a];
    for (int64_t b = 0; b < n_set; ++b) {
      if (is_nbr(P, xi, x + 3 * (int64_t)ids[b])) {
        if (tot >= cap) return -1;
        nbr[tot++] = ids[b];
      }
    }
  }
  off[n_set] = tot;
  return tot;
}

/* Grid of the cell-linked list: cell size 2h over [lo, hi]; dims = floor(L/(2h)) + 1. */
void orc_grid_dims(const orc_params* P, int64_t dims[3], double* inv) {
  *inv = 1.0 / (2.0 * P->h);
  for (int a = 0; a < 3; ++a) dims[a] = (int64_t)floor((P->hi[a] - P->lo[a]) * (*inv)) + 1;
}

/* Integer cell coordinate along one axis: floor((x - lo) * inv), clamped. */
static int64_t cell_coord(double x, double lo, double inv, int64_t dim) {
  double t = floor((x - lo) * inv);
  if (t < 0.0) return 0;
  if (t > (double)(dim - 1)) return dim - 1;
  return (int64_t)t;
}

/* Cell of a stored position, clamped to the grid: floor((x - lo) / (2h)) of the
 * FP32 absolute position, or the stored cell index. */
static void cell_of(const orc_params* P, const double* x, const int64_t dims[3], double inv, int64_t out[3]) {
  rep_t r;
  to_rep(P, x, &r);
  for (int a = 0; a < 3; ++a) {
    if (P->pos_mode == 1) {
      int64_t c = r.c[a];
      out[a] = c < 0 ? 0 : (c > dims[a] - 1 ? dims[a] - 1 : c);
    } else {
      out[a] = cell_coord(r.o[a], P->lo[a], inv, dims[a]);
    }
  }
}

/* Step 1 of Sec. 4.1: c = z * (Y * X) + y * X + x. */
void orc_cell_keys(const orc_params* P, int64_t n_set, const int32_t* ids, const double* x,
                   int64_t* keys) {
  int64_t dims[3]; double inv;
  orc_grid_dims(P, dims, &inv);
  for (int64_t a = 0; a < n_set; ++a) {
    int64_t c[3];
    cell_of(P, x + 3 * (int64_t)ids[a], dims, inv, c);
    keys[a] = c[2] * (dims[1] * dims[0]) + c[1] * dims[0] + c[0];
  }
}

typedef struct { int64_t key; int32_t id; } kv_t;
static int kv_cmp(const void* pa, const void* pb) {
  const kv_t* a = (const kv_t*)pa; const kv_t* b = (const kv_t*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

/* Step 2 of Sec. 4.1: sort by cell index, ties by ascending particle id.
 * Step 3: cellStart[c] = first sorted position of cell c, cellEnd[c] = one past
 * the last; an empty cell has cellStart = cellEnd = number of particles in
 * cells below c. Outputs: sorted ids, their keys, and start/end over all
 * M = X*Y*Z cells. */
void orc_sort_cells(const orc_params* P, int64_t n_set, const int32_t* ids, const double* x,
                    int32_t* sorted_ids, int64_t* sorted_keys, int64_t M,
                    int64_t* cell_start, int64_t* cell_end) {
  int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_set > 0 ? n_set : 1));
  kv_t* kv = (kv_t*)malloc(sizeof(kv_t) * (size_t)(n_set > 0 ? n_set : 1));
  orc_cell_keys(P, n_set, ids, x, keys);
  for (int64_t a = 0; a < n_set; ++a) { kv[a].key = keys[a]; kv[a].id = ids[a]; }
  qsort(kv, (size_t)n_set, sizeof(kv_t), kv_cmp);
  for (int64_t a = 0; a < n_set; ++a) { sorted_ids[a] = kv[a].id; sorted_keys[a] = kv[a].key; }
  if (cell_start && cell_end) {
    int64_t p = 0;
    for (int64_t c = 0; c < M; ++c) {
      while (p < n_set && kv[p].key < c) ++p;
      cell_start[c] = p;
      int64_t q = p;
      while (q < n_set && kv[q].key == c) ++q;
      cell_end[c] = q;
    }
  }
  free(kv); free(keys);
}

/* Step 4 of Sec. 4.1 (Algorithm 1): for each particle of the set, scan the 27
 * cells around its own and keep j with |x_i - x_j| < 2h. Lists are sorted by
 * id afterwards so that both search modes give identical sets in identical
 * order. Indexing of off/nbr is as in orc_neighbors_brute. */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t orc_neighbors_cells(const orc_params* P, int64_t n_set, const int32_t* ids,
                            const double* x, int64_t* off, int32_t* nbr, int64_t cap) {
  int64_t dims[3]; double inv;
  orc_grid_dims(P, dims, &inv);
  int64_t M = dims[0] * dims[1] * dims[2];
  int32_t* sid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_set > 0 ? n_set : 1));
  int64_t* skey = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_set > 0 ? n_set : 1));
  int64_t* cs = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
  int64_t* ce = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
  orc_sort_cells(P, n_set, ids, x, sid, skey, M, cs, ce);
  /* counts first (the paper precomputes offsets by a prefix sum of counts) */
  int64_t* cnt = (int64_t*)calloc((size_t)(n_set + 1), sizeof(int64_t));
  int64_t ret = 0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      int64_t s = 0;
      for (int64_t a = 0; a < n_set; ++a) { off[a] = s; s += cnt[a]; }
      off[n_set] = s;
      if (s > cap) { ret = -1; break; }
      ret = s;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t a = 0; a < n_set; ++a) {
      const double* xi = x + 3 * (int64_t)ids[a];
      int64_t c[3];
      cell_of(P, xi, dims, inv, c);
      int64_t count = 0;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dxx = -1; dxx <= 1; ++dxx) {
            int64_t q[3] = {c[0] + dxx, c[1] + dy, c[2] + dz};
            int skip = 0;
            for (int k = 0; k < 3; ++k) if (q[k] < 0 || q[k] >= dims[k]) skip = 1;
            if (skip) continue;
            int64_t cid = q[2] * (dims[1] * dims[0]) + q[1] * dims[0] + q[0];
            for (int64_t s = cs[cid]; s < ce[cid]; ++s) {
              int32_t j = sid[s];
              if (is_nbr(P, xi, x + 3 * (int64_t)j)) {
                if (pass == 1) nbr[off[a] + count] = j;
                ++count;
              }
            }
          }
      if (pass == 0) cnt[a] = count;
      else qsort(nbr + off[a], (size_t)count, sizeof(int32_t), cmp_i32);
    }
  }
  free(cnt); free(ce); free(cs); free(skey); free(sid);
  return ret;
}

/* ------------------------------------------------------- return mapping */
/* Pressure and equivalent shear stress of a symmetric tensor stored as
 * (xx, yy, zz, xy, xz, yz): p = -tr/3, tau = s + pI, taubar = sqrt(tau:tau / 2)
 * (Sec. 2.4, eq. trial_quantities). */
static void p_taubar(const double s[6], double* p, double* tb) {
  double pp = -(s[0] + s[1] + s[2]) / 3.0;
  double t0 = s[0] + pp, t1 = s[1] + pp, t2 = s[2] + pp;
  double dd = t0 * t0 + t1 * t1 + t2 * t2 + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  *p = pp; *tb = sqrt(0.5 * dd);
}

/* mu(I) of eq. muI, with the readings for the undefined cases:
 * gamma_dot < 0 is taken as 0; gamma_dot = 0 gives mu_s; p <= 0 gives mu_2. */
double orc_mu_I(const orc_params* P, double gamma_dot, double p) {
  if (gamma_dot < 0.0) gamma_dot = 0.0;
  if (gamma_dot == 0.0) return P->mu_s;
  if (p <= 0.0) return P->mu_2;
  double I = gamma_dot * P->grain_d * sqrt(P->rho0 / p);
  return P->mu_s + (P->mu_2 - P->mu_s) / (1.0 + P->I0 / I);
}

/* Which case of mu(I) applies (readings of the undefined cases): 0 gamma_dot
 * <= 0 (mu_s), 1 p <= 0 with gamma_dot > 0 (mu_2), 2 the interior formula. */
static int mu_case(double gamma_dot, double p) {
  if (!(gamma_dot > 0.0)) return 0;
  if (p <= 0.0) return 1;
  return 2;
}

/* Four-step return mapping (Sec. 2.4) of the elastic trial stress s_star, with
 * taubar^n taken from s_n (the stress at the start of the step). Writes the
 * corrected stress to out and, if mucase is not NULL, the mu(I) case of step 2
 * (-1 when step 1 ends the mapping). Returns the branch taken: 1 tension
 * cut-off, 3 admissible, 4 radial return. */
int orc_return_map_ex(const orc_params* P, const double s_star[6], const double s_n[6],
                      double out[6], int* mucase) {
  double G = P->E / (2.0 * (1.0 + P->nu));
  double ps, tbs, pn, tbn;
  p_taubar(s_star, &ps, &tbs);
  p_taubar(s_n, &pn, &tbn);
  if (mucase) *mucase = -1;
  /* step 1: p_cri = -c / mu_s; p* < p_cri (strict) gives zero stress */
  double p_cri = -P->cohesion / P->mu_s;
  if (ps < p_cri) { for (int k = 0; k < 6; ++k) out[k] = 0.0; return 1; }
  /* step 2: mu(I) with gamma_dot = (taubar* - taubar^n) / (G dt) */
  double gd = (tbs - tbn) / (G * P->dt);
  if (mucase) *mucase = mu_case(gd, ps);
  double mu = orc_mu_I(P, gd, ps);
  /* step 3: tau_max = mu p* + c (clamped at 0); keep if taubar* <= tau_max */
  double tmax = mu * ps + P->cohesion;
  if (tmax < 0.0) tmax = 0.0;
  if (tbs <= tmax) { for (int k = 0; k < 6; ++k) out[k] = s_star[k]; return 3; }
  /* step 4: radial return of the deviator, pressure unchanged */
  double f = tmax / tbs;
  out[0] = -ps + f * (s_star[0] + ps);
  out[1] = -ps + f * (s_star[1] + ps);
  out[2] = -ps + f * (s_star[2] + ps);
  out[3] = f * s_star[3];
  out[4] = f * s_star[4];
  out[5] = f * s_star[5];
  return 4;
}

int orc_return_map(const orc_params* P, const double s_star[6], const double s_n[6],
                   double out[6]) {
  return orc_return_map_ex(P, s_star, s_n, out, NULL);
}

/* ------------------------------------------------------------- rigid bodies */
typedef struct {
  double X[3], q[4], V[3], W[3], A[3], Al[3];
  int32_t has_acc;
  double half[3];
} orc_body;

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_R(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void cross(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ----------------------------------------------------------------- context */
typedef struct orc_ctx {
  orc_params P;
  double G, K, cs, m;           /* shear/bulk moduli, sound speed, particle mass */
  int64_t n_soil, n;            /* soil particles first, then markers */
  int32_t nb;
  orc_body* B;
  int32_t* body;                /* -1 for soil, body index for markers */
  double* local;                /* 3n, body-frame marker offsets */
  double *x, *u, *s, *rho;      /* y_n */
  double *xm, *um, *sm, *rhom;  /* y_mid */
  double *dx_, *du, *ds, *drho; /* stage rates */
  uint8_t* flag;                /* 0 inactive, 1 extended, 2 active */
  int32_t* proc; int64_t n_proc;
  int32_t* slot;                /* id -> index in proc, or -1 */
  int64_t* off; int32_t* nbr; int64_t nbr_cap, nbr_tot;
  int64_t step; double t;
  int64_t cap;                  /* capacity of the working arrays (policy only) */
  double* F; double* T;         /* per body, 3 each */
  double* as;                   /* 3n marker accelerations of the last stage 2 */
  int32_t* mat;                 /* material of each soil particle (0 = the parameters) */
  int8_t* branch;               /* per particle, the last step's return-mapping branch
                                   (1, 3, 4 as orc_return_map; 0 not updated) */
  int8_t* mucase;               /* and its mu(I) case (-1 when cut off) */
  int32_t n_mat;
  double* mat_tab;              /* per material: mu_s, mu_2, cohesion */
} orc_ctx;

void orc_destroy(orc_ctx* c);

orc_ctx* orc_create(const orc_params* P, int64_t n_soil, const double* pos, const double* vel,
                    const double* sig, const double* rho, int32_t nb, const int64_t* n_mark,
                    const double* marker_local, const double* half) {
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  c->P = *P;
  c->G = P->E / (2.0 * (1.0 + P->nu));
  c->K = P->E / (3.0 * (1.0 - 2.0 * P->nu));
  c->cs = sqrt(c->K / P->rho0);
  c->m = P->rho0 * P->dx * P->dx * P->dx;
  int64_t nm = 0;
  for (int b = 0; b < nb; ++b) nm += n_mark[b];
  c->n_soil = n_soil; c->n = n_soil + nm; c->nb = nb;
  int64_t n = c->n;
  c->B = (orc_body*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(orc_body));
  for (int b = 0; b < nb; ++b) {
    c->B[b].q[0] = 1.0;
    for (int k = 0; k < 3; ++k) c->B[b].half[k] = half ? half[3 * b + k] : 0.0;
  }
  size_t n3 = sizeof(double) * 3 * (size_t)n, n6 = sizeof(double) * 6 * (size_t)n,
         n1 = sizeof(double) * (size_t)n;
  c->body = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  c->local = (double*)calloc(1, n3);
  c->x = (double*)calloc(1, n3); c->u = (double*)calloc(1, n3);
  c->s = (double*)calloc(1, n6); c->rho = (double*)calloc(1, n1);
  c->xm = (double*)calloc(1, n3); c->um = (double*)calloc(1, n3);
  c->sm = (double*)calloc(1, n6); c->rhom = (double*)calloc(1, n1);
  c->dx_ = (double*)calloc(1, n3); c->du = (double*)calloc(1, n3);
  c->ds = (double*)calloc(1, n6); c->drho = (double*)calloc(1, n1);
  c->flag = (uint8_t*)calloc((size_t)n, 1);
  c->proc = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  c->slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  c->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  c->F = (double*)calloc(3 * (size_t)(nb > 0 ? nb : 1), sizeof(double));
  c->T = (double*)calloc(3 * (size_t)(nb > 0 ? nb : 1), sizeof(double));
  c->as = (double*)calloc(1, n3);
  c->mat = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  c->branch = (int8_t*)calloc((size_t)n, 1);
  c->mucase = (int8_t*)calloc((size_t)n, 1);
  c->n_mat = 1;
  c->mat_tab = (double*)malloc(3 * sizeof(double));
  c->mat_tab[0] = P->mu_s; c->mat_tab[1] = P->mu_2; c->mat_tab[2] = P->cohesion;
  for (int64_t i = 0; i < n_soil; ++i) {
    for (int k = 0; k < 3; ++k) {
      c->x[3 * i + k] = pos[3 * i + k];
      c->u[3 * i + k] = vel ? vel[3 * i + k] : 0.0;
    }
    for (int k = 0; k < 6; ++k) c->s[6 * i + k] = sig ? sig[6 * i + k] : 0.0;
    c->rho[i] = rho ? rho[i] : P->rho0;
    c->body[i] = -1;
  }
  int64_t i = n_soil;
  for (int b = 0; b < nb; ++b)
    for (int64_t k = 0; k < n_mark[b]; ++k, ++i) {
      c->body[i] = b;
      for (int a = 0; a < 3; ++a) c->local[3 * i + a] = marker_local[3 * (i - n_soil) + a];
      c->rho[i] = P->rho0;
    }
  c->nbr_cap = 0; c->nbr = NULL;
  c->cap = 0;
  return c;
}

void orc_destroy(orc_ctx* c) {
  if (!c) return;
  free(c->B); free(c->body); free(c->local);
  free(c->x); free(c->u); free(c->s); free(c->rho);
  free(c->xm); free(c->um); free(c->sm); free(c->rhom);
  free(c->dx_); free(c->du); free(c->ds); free(c->drho);
  free(c->flag); free(c->proc); free(c->slot); free(c->off); free(c->nbr);
  free(c->F); free(c->T); free(c->as); free(c->mat); free(c->mat_tab);
  free(c->branch); free(c->mucase);
  free(c);
}

/* Materials: per material (mu_s, mu_2, cohesion) of the return mapping
 * (Sec. 2.4), and the material of each soil particle. */
void orc_set_materials(orc_ctx* c, int32_t n_mat, const double* tab, const int32_t* mat) {
  free(c->mat_tab);
  c->n_mat = n_mat;
  c->mat_tab = (double*)malloc(3 * sizeof(double) * (size_t)n_mat);
  memcpy(c->mat_tab, tab, 3 * sizeof(double) * (size_t)n_mat);
  for (int64_t i = 0; i < c->n_soil; ++i) c->mat[i] = mat[i];
}

void orc_set_bodies(orc_ctx* c, int32_t nb, const double* X, const double* q, const double* V,
                    const double* W, const double* A, const double* Al) {
  for (int b = 0; b < nb && b < c->nb; ++b) {
    for (int k = 0; k < 3; ++k) {
      c->B[b].X[k] = X[3 * b + k];
      c->B[b].V[k] = V ? V[3 * b + k] : 0.0;
      c->B[b].W[k] = W ? W[3 * b + k] : 0.0;
      c->B[b].A[k] = A ? A[3 * b + k] : 0.0;
      c->B[b].Al[k] = Al ? Al[3 * b + k] : 0.0;
    }
    for (int k = 0; k < 4; ++k) c->B[b].q[k] = q[4 * b + k];
    c->B[b].has_acc = (A != NULL || Al != NULL);
  }
}

/* Marker world positions from the (frozen) body poses: x = X + R * local. */
static void place_markers(orc_ctx* c) {
  for (int64_t i = c->n_soil; i < c->n; ++i) {
    const orc_body* b = &c->B[c->body[i]];
    double R[9];
    quat_R(b->q, R);
    const double* l = c->local + 3 * i;
    for (int a = 0; a < 3; ++a)
      c->x[3 * i + a] = b->X[a] + ((R[3 * a] * l[0] + R[3 * a + 1] * l[1]) + R[3 * a + 2] * l[2]);
    for (int a = 0; a < 3; ++a) c->xm[3 * i + a] = c->x[3 * i + a];
  }
}

/* Activity flag of one position against all active boxes (Sec. 4.2 item 2):
 * inside a box (|local| <= half on every axis) -> Active (2); inside the box
 * grown by 2h on every local axis -> Extended-Active (1); else Inactive (0). */
int orc_flag_of(const orc_params* P, int32_t nb, const orc_body* B, const double* xw) {
  int best = 0;
  for (int b = 0; b < nb; ++b) {
    if (B[b].half[0] <= 0.0 && B[b].half[1] <= 0.0 && B[b].half[2] <= 0.0) continue;
    double R[9], d[3], l[3];
    quat_R(B[b].q, R);
    for (int a = 0; a < 3; ++a) d[a] = xw[a] - B[b].X[a];
    for (int a = 0; a < 3; ++a) l[a] = (R[a] * d[0] + R[3 + a] * d[1]) + R[6 + a] * d[2];
    int in = 1, ext = 1;
    for (int a = 0; a < 3; ++a) {
      double al = fabs(l[a]);
      if (!(al <= B[b].half[a])) in = 0;
      if (!(al <= B[b].half[a] + 2.0 * P->h)) ext = 0;
    }
    if (in) return 2;
    if (ext) best = 1;
  }
  return best;
}

/* Capacity policy of Sec. 4.2 item 3: grow to ceil(G * n) when n exceeds the
 * capacity; at steps that are multiples of S_I, shrink to n when n / cap < S. */
int64_t orc_capacity_next(int64_t cap, int64_t n_ae, int64_t step, double G, double S, int64_t S_I) {
  if (n_ae > cap) return (int64_t)ceil(G * (double)n_ae);
  if (S_I > 0 && step % S_I == 0 && cap > 0 && (double)n_ae / (double)cap < S) return n_ae;
  return cap;
}

/* Rebuild (Algorithms 2 and 3): activity (if t > t_delay), compaction into the
 * processed set, capacity policy, and the neighbour lists of the processed set. */
static int rebuild(orc_ctx* c) {
  const orc_params* P = &c->P;
  int64_t n = c->n;
  if (P->active_domains && c->t > P->t_delay) {
    /* activity is evaluated on the stored positions, as the neighbour test */
    for (int64_t i = 0; i < n; ++i) {
      rep_t r;
      double xf[3];
      to_rep(P, c->x + 3 * i, &r);
      rep_abs(P, &r, xf);
      c->flag[i] = (uint8_t)orc_flag_of(P, c->nb, c->B, xf);
    }
  } else {
    for (int64_t i = 0; i < n; ++i) c->flag[i] = 2;
  }
  c->n_proc = 0;
  for (int64_t i = 0; i < n; ++i) {
    c->slot[i] = -1;
    if (c->flag[i]) { c->slot[i] = (int32_t)c->n_proc; c->proc[c->n_proc++] = (int32_t)i; }
  }
  c->cap = orc_capacity_next(c->cap, c->n_proc, c->step, P->grow_G, P->shrink_S, P->shrink_interval);
  for (;;) {
    int64_t r = (P->nbr_mode == 1)
                    ? orc_neighbors_cells(P, c->n_proc, c->proc, c->x, c->off, c->nbr, c->nbr_cap)
                    : orc_neighbors_brute(P, c->n_proc, c->proc, c->x, c->off, c->nbr, c->nbr_cap);
    if (r >= 0) { c->nbr_tot = r; return 0; }
    c->nbr_cap = c->nbr_cap ? 2 * c->nbr_cap : 64 * (c->n_proc + 1);
    free(c->nbr);
    c->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)c->nbr_cap);
    if (!c->nbr) return -1;
  }
}

/* BCE extrapolation (Sec. 2.5.1) for every processed marker, from the fluid
 * particles of its list, at state (X, U, S, RHO). Adami velocity
 * u~ = sum u_f W / sum W, no-slip u_s = 2 u_body - u~; stress
 * s_s = [sum s_f W - ((g - a_s) . sum rho_f (x_s - x_f) W) I] / sum W.
 * With no fluid neighbour: u_s = u_body, s_s = 0. */
static void bce(orc_ctx* c, const double* X, double* U, double* S, const double* RHO) {
  const orc_params* P = &c->P;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t a = 0; a < c->n_proc; ++a) {
    int32_t i = c->proc[a];
    if (c->body[i] < 0) continue;
    const orc_body* b = &c->B[c->body[i]];
    double r[3], ub[3], as[3], w[3], tmp[3];
    for (int k = 0; k < 3; ++k) r[k] = X[3 * i + k] - b->X[k];
    cross(b->W, r, tmp);
    for (int k = 0; k < 3; ++k) ub[k] = b->V[k] + tmp[k];
    cross(b->W, tmp, w);                        /* centripetal w x (w x r) */
    if (b->has_acc) {
      cross(b->Al, r, tmp);
      for (int k = 0; k < 3; ++k) as[k] = b->A[k] + tmp[k] + w[k];
    } else {
      for (int k = 0; k < 3; ++k) as[k] = w[k];
    }
    double sw = 0.0, su[3] = {0, 0, 0}, ss[6] = {0, 0, 0, 0, 0, 0}, sr[3] = {0, 0, 0};
    for (int64_t e = c->off[a]; e < c->off[a + 1]; ++e) {
      int32_t j = c->nbr[e];
      if (c->body[j] >= 0) continue;
      double d[3];
      sep(P, X + 3 * (int64_t)i, X + 3 * (int64_t)j, d);
      double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double W = kern_W(P, rr);
      sw += W;
      for (int k = 0; k < 3; ++k) su[k] += U[3 * (int64_t)j + k] * W;
      for (int k = 0; k < 6; ++k) ss[k] += S[6 * (int64_t)j + k] * W;
      for (int k = 0; k < 3; ++k) sr[k] += RHO[j] * d[k] * W;
    }
    if (sw > 0.0) {
      double gdot = 0.0;
      for (int k = 0; k < 3; ++k) gdot += (P->g[k] - as[k]) * sr[k];
      for (int k = 0; k < 3; ++k) U[3 * (int64_t)i + k] = 2.0 * ub[k] - su[k] / sw;
      for (int k = 0; k < 6; ++k) S[6 * (int64_t)i + k] = ss[k] / sw;
      for (int k = 0; k < 3; ++k) S[6 * (int64_t)i + k] -= gdot / sw;
    } else {
      for (int k = 0; k < 3; ++k) U[3 * (int64_t)i + k] = ub[k];
      for (int k = 0; k < 6; ++k) S[6 * (int64_t)i + k] = 0.0;
    }
  }
}

/* sigma . v for a symmetric tensor in (xx, yy, zz, xy, xz, yz) order. */
static void sdot(const double s[6], const double v[3], double o[3]) {
  o[0] = s[0] * v[0] + s[3] * v[1] + s[4] * v[2];
  o[1] = s[3] * v[0] + s[1] * v[1] + s[5] * v[2];
  o[2] = s[4] * v[0] + s[5] * v[1] + s[2] * v[2];
}

/* Artificial viscosity contribution of one pair to a_i (eqs.
 * artificial_viscosity_bilateral / _unilateral), with the sign that makes
 * approaching pairs repel: + gamma h c_s m_j / rhobar (v.r)/(r^2 + xi^2) gradW. */
static void av_pair(const orc_ctx* c, const double v[3], const double d[3], double r2,
                    double rho_i, double rho_j, const double gw[3], double acc[3]) {
  const orc_params* P = &c->P;
  if (P->av_mode == 0) return;
  double vr = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
  if (P->av_mode == 2 && !(vr < 0.0)) return;
  double xi = P->av_xi_over_h * P->h;
  double rbar = 0.5 * (rho_i + rho_j);
  double f = P->av_gamma * P->h * c->cs * (c->m / rbar) * vr / (r2 + xi * xi);
  for (int k = 0; k < 3; ++k) acc[k] += f * gw[k];
}

/* Marker accelerations from the momentum equation over fluid neighbours only
 * (no body force), and the per-body force F = sum m a_s and torque
 * T = sum (x_s - X_b) x m a_s (Sec. 2.5.1). */
static void marker_forces(orc_ctx* c, const double* X, const double* U, const double* S,
                          const double* RHO) {
  const orc_params* P = &c->P;
  for (int b = 0; b < 3 * c->nb; ++b) { c->F[b] = 0.0; c->T[b] = 0.0; }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t a = 0; a < c->n_proc; ++a) {
    int32_t i = c->proc[a];
    double acc[3] = {0, 0, 0};
    if (c->body[i] >= 0) {
      for (int64_t e = c->off[a]; e < c->off[a + 1]; ++e) {
        int32_t j = c->nbr[e];
        if (c->body[j] >= 0) continue;
        double d[3], gw[3], t[3], ss[6], v[3];
        sep(P, X + 3 * (int64_t)i, X + 3 * (int64_t)j, d);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        gradW(P, d, sqrt(r2), gw);
        double Vj = c->m / RHO[j];
        for (int k = 0; k < 6; ++k) ss[k] = S[6 * (int64_t)i + k] + S[6 * (int64_t)j + k];
        sdot(ss, gw, t);
        for (int k = 0; k < 3; ++k) acc[k] += Vj * t[k] / RHO[i];
        for (int k = 0; k < 3; ++k) v[k] = U[3 * (int64_t)i + k] - U[3 * (int64_t)j + k];
        av_pair(c, v, d, r2, RHO[i], RHO[j], gw, acc);
      }
    }
    for (int k = 0; k < 3; ++k) c->as[3 * (int64_t)i + k] = acc[k];
  }
  /* sequential, id-ordered body sums */
  for (int64_t a = 0; a < c->n_proc; ++a) {
    int32_t i = c->proc[a];
    int b = c->body[i];
    if (b < 0) continue;
    double f[3], r[3], tq[3];
    for (int k = 0; k < 3; ++k) { f[k] = c->m * c->as[3 * (int64_t)i + k]; r[k] = X[3 * (int64_t)i + k] - c->B[b].X[k]; }
    cross(r, f, tq);
    for (int k = 0; k < 3; ++k) { c->F[3 * b + k] += f[k]; c->T[3 * b + k] += tq[k]; }
  }
}

/* Right-hand side for every Active soil particle at state (X, U, S, RHO):
 * L = sum_j V_j (u_j - u_i) (x) gradW  (F2, (L)_ab = du_a/dx_b)
 * drho/dt = -rho_i tr L                                      (continuity_dis)
 * du/dt   = (1/rho_i) sum_j V_j (s_i + s_j) . gradW + g + Pi  (momentum_dis, F3)
 * ds/dt   = Om s - s Om + 2G (D - tr D / 3 I) + bulk K tr D I (stress_rate_dis)
 * with D = (L + L^T)/2, Om = (L - L^T)/2 (spin of eq. stress_rate_jaumann). */
static void rhs(orc_ctx* c, const double* X, const double* U, const double* S, const double* RHO) {
  const orc_params* P = &c->P;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t a = 0; a < c->n_proc; ++a) {
    int32_t i = c->proc[a];
    if (c->body[i] >= 0 || c->flag[i] != 2) continue;
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, acc[3] = {0, 0, 0};
    const double* si = S + 6 * (int64_t)i;
    for (int64_t e = c->off[a]; e < c->off[a + 1]; ++e) {
      int32_t j = c->nbr[e];
      double d[3], gw[3], t[3], ss[6], du_[3], v[3];
      sep(P, X + 3 * (int64_t)i, X + 3 * (int64_t)j, d);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      gradW(P, d, sqrt(r2), gw);
      double Vj = c->m / RHO[j];
      for (int k = 0; k < 3; ++k) du_[k] = U[3 * (int64_t)j + k] - U[3 * (int64_t)i + k];
      for (int aa = 0; aa < 3; ++aa)
        for (int bb = 0; bb < 3; ++bb) L[3 * aa + bb] += Vj * du_[aa] * gw[bb];
      for (int k = 0; k < 6; ++k) ss[k] = si[k] + S[6 * (int64_t)j + k];
      sdot(ss, gw, t);
      for (int k = 0; k < 3; ++k) acc[k] += Vj * t[k] / RHO[i];
      for (int k = 0; k < 3; ++k) v[k] = -du_[k];   /* v_ij = u_i - u_j */
      av_pair(c, v, d, r2, RHO[i], RHO[j], gw, acc);
    }
    double trD = L[0] + L[4] + L[8];
    double D[9], Om[9];
    for (int aa = 0; aa < 3; ++aa)
      for (int bb = 0; bb < 3; ++bb) {
        D[3 * aa + bb] = 0.5 * (L[3 * aa + bb] + L[3 * bb + aa]);
        Om[3 * aa + bb] = 0.5 * (L[3 * aa + bb] - L[3 * bb + aa]);
      }
    double Sm[9] = {si[0], si[3], si[4], si[3], si[1], si[5], si[4], si[5], si[2]};
    double R[9];
    for (int aa = 0; aa < 3; ++aa)
      for (int bb = 0; bb < 3; ++bb) {
        double os = 0.0, so = 0.0;
        for (int k = 0; k < 3; ++k) {
          os += Om[3 * aa + k] * Sm[3 * k + bb];
          so += Sm[3 * aa + k] * Om[3 * k + bb];
        }
        double iso = (aa == bb) ? (P->bulk_coeff * c->K * trD - 2.0 * c->G * trD / 3.0) : 0.0;
        R[3 * aa + bb] = os - so + 2.0 * c->G * D[3 * aa + bb] + iso;
      }
    c->drho[i] = -RHO[i] * trD;
    for (int k = 0; k < 3; ++k) {
      c->du[3 * (int64_t)i + k] = acc[k] + P->g[k];
      c->dx_[3 * (int64_t)i + k] = U[3 * (int64_t)i + k];
    }
    double* dsi = c->ds + 6 * (int64_t)i;
    dsi[0] = R[0]; dsi[1] = R[4]; dsi[2] = R[8]; dsi[3] = R[1]; dsi[4] = R[2]; dsi[5] = R[5];
  }
}

/* One explicit-midpoint RK2 step (Sec. 2.3) with the return mapping after the
 * full step (Sec. 2.4). Extended-Active particles are read but never written;
 * markers are not integrated. Forces come from the stage-2 evaluation. */
static int one_step(orc_ctx* c) {
  const orc_params* P = &c->P;
  place_markers(c);
  if (c->step % P->ps_freq == 0)
    if (rebuild(c)) return -1;
  double h2 = 0.5 * P->dt;
  /* stage 1 at y_n */
  bce(c, c->x, c->u, c->s, c->rho);
  rhs(c, c->x, c->u, c->s, c->rho);
  for (int64_t i = 0; i < c->n; ++i) {
    int upd = (c->body[i] < 0 && c->flag[i] == 2);
    for (int k = 0; k < 3; ++k) {
      c->xm[3 * i + k] = upd ? c->x[3 * i + k] + h2 * c->dx_[3 * i + k] : c->x[3 * i + k];
      c->um[3 * i + k] = upd ? c->u[3 * i + k] + h2 * c->du[3 * i + k] : c->u[3 * i + k];
    }
    for (int k = 0; k < 6; ++k)
      c->sm[6 * i + k] = upd ? c->s[6 * i + k] + h2 * c->ds[6 * i + k] : c->s[6 * i + k];
    c->rhom[i] = upd ? c->rho[i] + h2 * c->drho[i] : c->rho[i];
  }
  /* stage 2 at y_mid */
  bce(c, c->xm, c->um, c->sm, c->rhom);
  marker_forces(c, c->xm, c->um, c->sm, c->rhom);
  rhs(c, c->xm, c->um, c->sm, c->rhom);
  for (int64_t i = 0; i < c->n; ++i) {
    c->branch[i] = 0;
    c->mucase[i] = -1;
    if (!(c->body[i] < 0 && c->flag[i] == 2)) continue;
    for (int k = 0; k < 3; ++k) {
      c->x[3 * i + k] += P->dt * c->dx_[3 * i + k];
      c->u[3 * i + k] += P->dt * c->du[3 * i + k];
    }
    double sn[6], sstar[6];
    for (int k = 0; k < 6; ++k) { sn[k] = c->s[6 * i + k]; sstar[k] = sn[k] + P->dt * c->ds[6 * i + k]; }
    orc_params Pm = *P;             /* the return mapping with the particle's material */
    const double* mt = c->mat_tab + 3 * c->mat[i];
    Pm.mu_s = mt[0]; Pm.mu_2 = mt[1]; Pm.cohesion = mt[2];
    int mc = -1;
    c->branch[i] = (int8_t)orc_return_map_ex(&Pm, sstar, sn, c->s + 6 * i, &mc);
    c->mucase[i] = (int8_t)mc;
    c->rho[i] += P->dt * c->drho[i];
  }
  /* marker values of the midpoint are what the step last computed */
  for (int64_t i = c->n_soil; i < c->n; ++i) {
    for (int k = 0; k < 3; ++k) c->u[3 * i + k] = c->um[3 * i + k];
    for (int k = 0; k < 6; ++k) c->s[6 * i + k] = c->sm[6 * i + k];
  }
  c->step += 1;
  c->t = (double)c->step * P->dt;
  return 0;
}

int orc_step(orc_ctx* c, int64_t n_steps) {
  for (int64_t k = 0; k < n_steps; ++k)
    if (one_step(c)) return -1;
  return 0;
}

/* One evaluation of the right-hand side at the current state, after a rebuild
 * from the current positions (for closed-form checks). Fills, for all n
 * particles: drho, du (including g), ds for Active soil particles; for
 * processed markers, u and s of the extrapolation and the acceleration a_s. */
int orc_eval_rhs(orc_ctx* c, double* drho, double* du, double* ds, double* mu, double* ms,
                 double* mas) {
  place_markers(c);
  if (rebuild(c)) return -1;
  for (int64_t i = 0; i < c->n; ++i) {
    c->drho[i] = 0.0;
    for (int k = 0; k < 3; ++k) c->du[3 * i + k] = 0.0;
    for (int k = 0; k < 6; ++k) c->ds[6 * i + k] = 0.0;
  }
  bce(c, c->x, c->u, c->s, c->rho);
  marker_forces(c, c->x, c->u, c->s, c->rho);
  rhs(c, c->x, c->u, c->s, c->rho);
  memcpy(drho, c->drho, sizeof(double) * (size_t)c->n);
  memcpy(du, c->du, sizeof(double) * 3 * (size_t)c->n);
  memcpy(ds, c->ds, sizeof(double) * 6 * (size_t)c->n);
  if (mu) memcpy(mu, c->u, sizeof(double) * 3 * (size_t)c->n);
  if (ms) memcpy(ms, c->s, sizeof(double) * 6 * (size_t)c->n);
  if (mas) memcpy(mas, c->as, sizeof(double) * 3 * (size_t)c->n);
  return 0;
}

/* Fluid acceleration contributed by the markers of body `b` alone, at the
 * current state and lists (for the action-reaction check of body forces). */
void orc_fluid_acc_from_body(orc_ctx* c, int32_t bsel, double* out) {
  const orc_params* P = &c->P;
  const double *X = c->x, *U = c->u, *S = c->s, *RHO = c->rho;
  for (int64_t i = 0; i < 3 * c->n; ++i) out[i] = 0.0;
  for (int64_t a = 0; a < c->n_proc; ++a) {
    int32_t i = c->proc[a];
    if (c->body[i] >= 0) continue;
    double acc[3] = {0, 0, 0};
    for (int64_t e = c->off[a]; e < c->off[a + 1]; ++e) {
      int32_t j = c->nbr[e];
      if (c->body[j] != bsel) continue;
      double d[3], gw[3], t[3], ss[6], v[3];
      sep(P, X + 3 * (int64_t)i, X + 3 * (int64_t)j, d);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      gradW(P, d, sqrt(r2), gw);
      double Vj = c->m / RHO[j];
      for (int k = 0; k < 6; ++k) ss[k] = S[6 * (int64_t)i + k] + S[6 * (int64_t)j + k];
      sdot(ss, gw, t);
      for (int k = 0; k < 3; ++k) acc[k] += Vj * t[k] / RHO[i];
      for (int k = 0; k < 3; ++k) v[k] = U[3 * (int64_t)i + k] - U[3 * (int64_t)j + k];
      av_pair(c, v, d, r2, RHO[i], RHO[j], gw, acc);
    }
    for (int k = 0; k < 3; ++k) out[3 * (int64_t)i + k] = acc[k];
  }
}

/* ------------------------------------------------------------ accessors */
int64_t orc_n(const orc_ctx* c) { return c->n; }
int64_t orc_n_proc(const orc_ctx* c) { return c->n_proc; }
int64_t orc_nbr_total(const orc_ctx* c) { return c->nbr_tot; }
int64_t orc_capacity(const orc_ctx* c) { return c->cap; }
int64_t orc_step_count(const orc_ctx* c) { return c->step; }
double orc_mass(const orc_ctx* c) { return c->m; }

void orc_get_state(const orc_ctx* c, double* x, double* u, double* s, double* rho) {
  if (x) memcpy(x, c->x, sizeof(double) * 3 * (size_t)c->n);
  if (u) memcpy(u, c->u, sizeof(double) * 3 * (size_t)c->n);
  if (s) memcpy(s, c->s, sizeof(double) * 6 * (size_t)c->n);
  if (rho) memcpy(rho, c->rho, sizeof(double) * (size_t)c->n);
}

void orc_set_state(orc_ctx* c, const double* x, const double* u, const double* s, const double* rho) {
  for (int64_t i = 0; i < c->n_soil; ++i) {
    if (x) for (int k = 0; k < 3; ++k) c->x[3 * i + k] = x[3 * i + k];
    if (u) for (int k = 0; k < 3; ++k) c->u[3 * i + k] = u[3 * i + k];
    if (s) for (int k = 0; k < 6; ++k) c->s[6 * i + k] = s[6 * i + k];
    if (rho) c->rho[i] = rho[i];
  }
}

void orc_get_forces(const orc_ctx* c, double* F, double* T) {
  memcpy(F, c->F, sizeof(double) * 3 * (size_t)c->nb);
  memcpy(T, c->T, sizeof(double) * 3 * (size_t)c->nb);
}

void orc_get_flags(const orc_ctx* c, uint8_t* flags) { memcpy(flags, c->flag, (size_t)c->n); }

/* Return-mapping branch and mu(I) case of every particle in the last step. */
void orc_get_branches(const orc_ctx* c, int8_t* branch, int8_t* mucase) {
  if (branch) memcpy(branch, c->branch, (size_t)c->n);
  if (mucase) memcpy(mucase, c->mucase, (size_t)c->n);
}

/* Stored form of one position (pos_mode 1: integer cell and FP32 offset; pos_mode
 * 0: the FP32 coordinate in o, c = 0), for checks of the representation. */
void orc_to_rep(const orc_params* P, const double* x, int64_t* c, double* o) {
  rep_t r;
  to_rep(P, x, &r);
  for (int a = 0; a < 3; ++a) { c[a] = r.c[a]; o[a] = r.o[a]; }
}

/* Processed set (ascending ids) and its lists, as of the last rebuild. */
void orc_get_lists(const orc_ctx* c, int32_t* proc, int64_t* off, int32_t* nbr) {
  if (proc) memcpy(proc, c->proc, sizeof(int32_t) * (size_t)c->n_proc);
  if (off) memcpy(off, c->off, sizeof(int64_t) * (size_t)(c->n_proc + 1));
  if (nbr) memcpy(nbr, c->nbr, sizeof(int32_t) * (size_t)c->nbr_tot);
}

/* Positions of all particles (markers placed from the current poses). */
void orc_positions(orc_ctx* c, double* x) {
  place_markers(c);
  memcpy(x, c->x, sizeof(double) * 3 * (size_t)c->n);
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
