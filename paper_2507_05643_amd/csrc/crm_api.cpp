// Host side of the libcrm C ABI (include/crm.h): validation, device memory,
// the rebuild pipeline of Alg. 3 (activity, compaction, capacity policy, cell
// hashing, sort, neighbour lists) and the two-stage step of Sec. 2.3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "crm.h"
#include "crm_internal.h"

using crm::Body;
using crm::Grid;
using crm::Phys;
using crm::CPlanes;
using crm::Planes;

namespace {

std::string g_init_error = "no error";

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct crm_ctx {
  crm_params prm{};
  int device = 0;
  hipStream_t stream = nullptr;
  crm_alloc_fn alloc = nullptr;
  crm_free_fn free_fn = nullptr;
  void* user = nullptr;
  bool poisoned = false;
  bool noalloc = false;        // set during a call that must not allocate
  void* scratch = nullptr;     // this device's static scratch array (crm_step_noalloc)
  std::string err = "no error";

  int64_t n_soil = 0, n_mark = 0, n_total = 0;
  int32_t nb = 0;
  Grid grid{};
  Phys phys{};
  int64_t M = 0;
  Grid wgrid{};                // the grid of the last rebuild: the domain's, or a window of it
  int64_t Mw = 0;              // its cells
  bool ad_on = false;  // last rebuild used the activity flags

  // master store (by particle id), four planes of float4
  float4 *m_a = nullptr, *m_b = nullptr, *m_c = nullptr, *m_d = nullptr;
  float4* local = nullptr;     // markers: (lx, ly, lz, body bits)
  uint8_t* flags = nullptr;
  uint32_t* m_key = nullptr;      // the activity pre-test's compact positions (active domains only)
  // launch order of the stage kernels' soil blocks (block_order), sized for the domain's grid
  int32_t* bperm = nullptr;
  uint32_t *ord_cnt = nullptr, *ord_first = nullptr, *ord_base = nullptr, *ord_scan = nullptr;
  int64_t ord_cap = 0;
  // active-domain flags from an index by coarse cell (active domains, activity_scan 0)
  bool ix_on = false;             // index allocated
  bool ix_valid = false;          // every particle not on the moved list is where the index lists it
  bool flags_valid = false;       // flags hold exactly the last compaction's ids (proc_ids, d_counts[0])
  bool ix_used = false;           // this rebuild's flags came from the index
  int32_t ix_cd[3] = {0, 0, 0};
  int64_t ix_M = 0;
  uint32_t* ix_start = nullptr;   // ix_M + 1
  uint32_t* ix_fill = nullptr;    // ix_M
  uint32_t* ix_scan = nullptr;
  int32_t* ix_ids = nullptr;      // n_total
  uint32_t* ix_visit = nullptr;   // ix_M
  uint32_t* h_visit_pin = nullptr;  // ix_M (pinned host: the visit list's upload)
  uint8_t* moved = nullptr;       // flags_padded(n_total)
  int32_t* mlist = nullptr;       // mcap; its count in d_counts[6]
  int64_t mcap = 0;
  std::vector<uint32_t> h_visit;
  std::vector<Body> ix_bodies;    // body poses when the index was built
  std::vector<uint8_t> ix_moving; // bodies whose markers are on the moved list
  int32_t* proc_ids = nullptr;
  Body* d_bodies = nullptr;
  float4* d_mat = nullptr;     // material table
  int32_t n_mat = 1;
  std::vector<uint16_t> h_mat; // material of each soil particle (empty: all 0)
  std::vector<float4> h_mattab;  // material table as uploaded (n_mat rows)
  std::vector<Body> h_bodies;
  std::vector<Body> h_bodies_next;  // validation buffer of crm_set_bodies (nb, kept allocated)
  std::vector<int64_t> h_nmark;  // markers per body
  std::vector<int64_t> h_bstart; // first marker (relative id) of each body, nb + 1
  // host buffers of the force-sum plan, sized once at crm_init (a rebuild
  // step allocates no host memory)
  std::vector<int64_t> plan_lo, plan_hi, plan_r;
  std::vector<int32_t> plan_first;
  double* d_fmap = nullptr;       // device alias of h_fpin: the body sums are written there
  uint32_t* ctmp = nullptr;    // compaction scratch (n_total sized)

  // cell grid
  uint32_t* cell_cnt = nullptr;
  uint32_t* cell_start = nullptr;
  uint32_t* cell_tmp = nullptr;

  // working set (capacity `cap`)
  int64_t cap = 0;
  Planes A{}, B{};
  float4* pos4 = nullptr;
  int4* cpos = nullptr;          // cells of the sorted slots (cell-offset positions)
  int32_t* slot_id = nullptr;
  int32_t* slot_k = nullptr;     // processed index (position in the processed id list)
  uint32_t *skey = nullptr, *key = nullptr, *rank = nullptr, *tmp = nullptr;
  uint64_t* tmpx = nullptr;     // x order keys beside tmp (sort inside cells)
  int32_t *frows = nullptr, *mrows = nullptr;
  int32_t* near = nullptr;       // marker rows (indices into mrows) with soil neighbours
  crm::NearRow* nrow = nullptr;  // their slots and list ranges, for the BCE passes
  int64_t n_near = 0;
  uint32_t *cnt_f = nullptr, *cnt_m = nullptr;
  uint64_t *off_f = nullptr, *off_m = nullptr, *wtmp = nullptr;
  uint32_t *stash_f = nullptr, *stash_m = nullptr;  // count-pass scratch of the lists
  uint32_t* tabs = nullptr;       // LDS tile tables of the soil-row blocks
  int32_t tile_cfg = CRM_TILE_SMALL;  // LDS tile configuration of the soil stages

  // neighbour entries
  uint32_t* nbr_f = nullptr;
  int64_t nbr_f_cap = 0;
  uint16_t* tix_f = nullptr;     // tile positions of the soil entries (nbr_f_cap)
  int64_t tix_f_cap = 0;
  // nbr_f lacks the slots of the staged blocks with at most this many tile
  // records (the stages read those blocks from their tiles; 0: nbr_f complete)
  uint32_t nbr_skip = 0;
  bool full_lists = false;        // rebuilds write every slot (reverse sweep)
  uint32_t* nbr_m = nullptr;
  int64_t nbr_m_cap = 0;

  double* contrib = nullptr;     // per marker id: force and torque on its body (6 FP64)
  int64_t* d_bstart = nullptr;   // first marker id (relative) of each body, nb + 1
  crm::SegPlan body_plan;        // chunked per-body force sums over the processed markers
  int64_t plan_cap = 0;          // chunk capacity of body_plan
  int64_t* d_branges = nullptr;  // per body: first processed-marker rank (nb + 1)
  bool plan_all = false;         // body_plan covers all markers (every particle processed)
  int64_t kbase = 0;             // rank of the first processed marker in the processed list
  std::vector<Body> placed;      // body poses of the markers' last placement in the master store
  std::vector<Body> wplaced;     // body states of the markers' last placement in the working set
  bool wplaced_ok = false;       // wplaced holds them (else every body counts as moved)
  bool place_all = true;         // place every body's markers at the next placement
  // Verlet lists (skin > 0): steps of the last rebuild, largest squared
  // displacement since (device word, pinned mirror, event of its copy)
  int64_t last_rebuild = 0;
  uint32_t* d_disp = nullptr;
  uint32_t* h_disp = nullptr;
  // co-simulation exchange: body states up through pinned staging; forces and
  // torques (6 per body) written by the device into mapped pinned memory;
  // each with its completion event
  Body* h_bpin = nullptr;
  double* h_fpin = nullptr;
  hipEvent_t bpin_ev = nullptr, fpin_ev = nullptr;
  int64_t fpin_step = -1;         // the counters mark the body sums of the step that leaves c->step at this value
  volatile uint64_t* h_fseq = nullptr;   // per body: reductions written (host view, after the sums in h_fpin)
  uint64_t* d_fseq = nullptr;            // device alias of h_fseq
  uint64_t fseq = 0;                     // reductions enqueued
  bool bpin_pending = false;
  hipEvent_t disp_ev = nullptr;
  bool disp_pending = false;
  uint64_t* d_counts = nullptr;   // [0] n_proc [1] soil rows [2] marker rows [3] f entries [4] m entries
                                 // [5] marker rows with soil neighbours
  uint64_t* h_counts = nullptr;   // pinned mirror

  int64_t n_proc = 0, n_frows = 0, n_mrows = 0, ent_f = 0, ent_m = 0;
  int64_t step = 0, rebuilds = 0;
  bool working_valid = false;
  bool force_rebuild = true;
  bool stepped = false;

  // replay of the per-step kernels as one hipGraph
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr, graph2 = nullptr;   // a step's kernels up to the body sums, then stage 2
  hipGraphExec_t gexec = nullptr, gexec2 = nullptr;
  std::vector<const void*> graph_key;

  // profiling: event pairs per kernel class
  bool prof = false;
  uint32_t prof_mask = 0;        // kernel classes timed while profiling (bit k = class k)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_marks;

  // reverse mode: a recorded run of steps (crm_record) and its adjoint sweep
  bool recording = false;
  bool rec_valid = false;
  int32_t rec_n = 0;               // recorded steps
  int64_t rec_step0 = 0;           // step counter at the start of the record
  std::vector<int64_t> rec_seg;    // first step (relative) of each rebuild segment
  std::vector<Body> rec_bodies;    // the body table the record ran with
  float4* rec_snap = nullptr;      // master planes at each segment start (4 x n_total each)
  int64_t rec_snap_cap = 0;        // segments the snapshot buffer holds
  double* rec_forces = nullptr;    // per recorded step: the bodies' force and torque (6 nb)

  std::vector<Buf> owned;
};

namespace {

crm_status fail(crm_ctx* c, crm_status st, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (st == CRM_E_DEVICE || st == CRM_E_NONFINITE) c->poisoned = true;
  } else {
    g_init_error = msg;
  }
  return st;
}

void* dalloc(crm_ctx* c, size_t bytes) {
  if (c->noalloc) return nullptr;   // a call that must not allocate
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (c->alloc) {
    p = c->alloc(bytes, c->user, (void*)c->stream);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->owned.push_back(Buf{p, bytes});
  return p;
}

void dfree(crm_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->owned.size(); ++i) {
    if (c->owned[i].p == p) {
      c->owned.erase(c->owned.begin() + (long)i);
      break;
    }
  }
  if (c->free_fn)
    c->free_fn(p, c->user, (void*)c->stream);
  else
    (void)hipFree(p);
}

template <typename T>
bool alloc_n(crm_ctx* c, T*& p, int64_t n) {
  p = (T*)dalloc(c, sizeof(T) * (size_t)(n > 0 ? n : 1));
  return p != nullptr;
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

std::string check_params(const crm_params* p) {
  if (!p) return "params is NULL";
  if (p->abi_version != CRM_ABI_VERSION) return "abi_version mismatch";
  if (p->pos_mode > 1) return "pos_mode must be CRM_POS_FP32 or CRM_POS_CELL_OFFSET";
  if (p->kernel > 1) return "kernel must be CRM_KERNEL_CUBIC or CRM_KERNEL_WENDLAND";
  if (p->activity_scan > 1) return "activity_scan must be 0 or 1";
  if (p->moved_cap < 0) return "moved_cap must be >= 0";
  if (!(std::isfinite(p->skin) && p->skin >= 0.0)) return "skin must be >= 0";
  auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
  if (!pos(p->dx)) return "dx must be > 0";
  if (!pos(p->h)) return "h must be > 0";
  if (!pos(p->dt)) return "dt must be > 0";
  if (!finite3(p->gravity)) return "gravity must be finite";
  if (!pos(p->rho0)) return "rho0 must be > 0";
  if (!pos(p->E)) return "E must be > 0";
  if (!(std::isfinite(p->nu) && p->nu >= 0.0 && p->nu < 0.5)) return "nu must be in [0, 0.5)";
  if (!pos(p->mu_s)) return "mu_s must be > 0";
  if (!(std::isfinite(p->mu_2) && p->mu_2 >= 0.0)) return "mu_2 must be >= 0";
  if (!pos(p->I0)) return "I0 must be > 0";
  if (!pos(p->grain_d)) return "grain_d must be > 0";
  if (!(std::isfinite(p->cohesion) && p->cohesion >= 0.0)) return "cohesion must be >= 0";
  if (p->av_mode > 2) return "av_mode must be 0, 1 or 2";
  if (!(std::isfinite(p->av_gamma) && p->av_gamma >= 0.0)) return "av_gamma must be >= 0";
  if (!pos(p->av_xi_over_h)) return "av_xi_over_h must be > 0";
  for (int a = 0; a < 3; ++a)
    if (!(std::isfinite(p->domain_lo[a]) && std::isfinite(p->domain_hi[a]) && p->domain_hi[a] > p->domain_lo[a]))
      return "domain_hi must exceed domain_lo on every axis";
  if (p->ps_freq < 1) return "ps_freq must be >= 1";
  if (p->active_domains > 1) return "active_domains must be 0 or 1";
  if (!std::isfinite(p->t_delay)) return "t_delay must be finite";
  if (!(std::isfinite(p->grow_G) && p->grow_G >= 1.0)) return "grow_G must be >= 1";
  if (!(std::isfinite(p->shrink_S) && p->shrink_S > 0.0 && p->shrink_S <= 1.0)) return "shrink_S must be in (0, 1]";
  if (p->shrink_interval < 1) return "shrink_interval must be >= 1";
  if (!std::isfinite(p->bulk_coeff)) return "bulk_coeff must be finite";
  return "";
}

// FP64 coordinate <-> cell index + FP32 offset (cell-offset positions).
void to_cell(double x, double lo, double inv, double S, int32_t& c, float& o) {
#pragma clang fp contract(off)
  const double t = x - lo;
  const double cc = std::floor(t * inv);
  c = (int32_t)cc;
  o = (float)(t - cc * S);
}

double from_cell(int32_t c, float o, double lo, double S) {
#pragma clang fp contract(off)
  return (lo + (double)c * S) + (double)o;
}

// Stored position (a.xyz, d.zw) of a host FP64 position.
void host_store_pos(const crm_ctx* c, const double* x, float4& a, float4& d) {
  if (c->grid.cell) {
    int32_t q[3];
    float o[3];
    for (int k = 0; k < 3; ++k) to_cell(x[k], c->grid.lo[k], c->grid.inv, c->grid.S, q[k], o[k]);
    a.x = o[0]; a.y = o[1]; a.z = o[2];
    uint32_t cx = (uint32_t)q[0], yz = crm::pack_yz(q[1], q[2]);
    std::memcpy(&d.z, &cx, 4);
    std::memcpy(&d.w, &yz, 4);
  } else {
    a.x = (float)x[0]; a.y = (float)x[1]; a.z = (float)x[2];
  }
}

void host_abs_pos(const crm_ctx* c, const float4& a, const float4& d, double* x) {
  if (c->grid.cell) {
    uint32_t cx, yz;
    std::memcpy(&cx, &d.z, 4);
    std::memcpy(&yz, &d.w, 4);
    x[0] = from_cell((int32_t)cx, a.x, c->grid.lo[0], c->grid.S);
    x[1] = from_cell(crm::unpack_y(yz), a.y, c->grid.lo[1], c->grid.S);
    x[2] = from_cell(crm::unpack_z(yz), a.z, c->grid.lo[2], c->grid.S);
  } else {
    x[0] = a.x; x[1] = a.y; x[2] = a.z;
  }
}

void quat_to_R(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, CRM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The capacity-sized arrays of the working set, with their element sizes and
// counts at capacity cap.
struct WorkBuf {
  void** field;
  size_t elem;
  int64_t count;
};

std::vector<WorkBuf> work_buffers(crm_ctx* c, int64_t cap) {
  auto f = [](auto*& p) { return reinterpret_cast<void**>(&p); };
  return {{f(c->A.a), sizeof(float4), cap},   {f(c->A.b), sizeof(float4), cap},   {f(c->A.c), sizeof(float4), cap},
          {f(c->A.d), sizeof(float4), cap},   {f(c->B.a), sizeof(float4), cap},   {f(c->B.b), sizeof(float4), cap},
          {f(c->B.c), sizeof(float4), cap},   {f(c->B.d), sizeof(float4), cap},   {f(c->pos4), sizeof(float4), cap},
          {f(c->cpos), sizeof(int4), c->grid.cell ? cap : 1},
          {f(c->slot_id), 4, cap},            {f(c->slot_k), 4, cap},             {f(c->skey), 4, cap},
          {f(c->key), 4, cap},                {f(c->rank), 4, cap},               {f(c->tmp), 4, cap},
          {f(c->tmpx), 8, cap},               {f(c->frows), 4, cap},              {f(c->mrows), 4, cap},
          {f(c->near), 4, cap},               {f(c->nrow), sizeof(crm::NearRow), cap},
          {f(c->cnt_f), 4, cap},              {f(c->cnt_m), 4, cap},              {f(c->off_f), 8, cap + 1},
          {f(c->off_m), 8, cap + 1},          {f(c->wtmp), 8, (int64_t)crm::scan_tmp_elems(cap)},
          {f(c->stash_f), 4, (int64_t)crm::stash_elems(cap)},
          {f(c->stash_m), 4, (int64_t)crm::stash_elems(cap)},
          {f(c->tabs), 4, crm::tile_table_words(cap)}};
}

// New working arrays of capacity cap. All of them are taken before the old
// ones are released, so a failed allocation leaves the context as it was.
crm_status realloc_working(crm_ctx* c, int64_t cap) {
  std::vector<WorkBuf> bufs = work_buffers(c, cap);
  std::vector<void*> fresh(bufs.size(), nullptr);
  for (size_t i = 0; i < bufs.size(); ++i) {
    fresh[i] = dalloc(c, bufs[i].elem * (size_t)(bufs[i].count > 0 ? bufs[i].count : 1));
    if (!fresh[i]) {
      for (size_t j = 0; j < i; ++j) dfree(c, fresh[j]);
      return fail(c, CRM_E_NOMEM, c->noalloc ? "the working set must grow (a call that may allocate is needed)"
                                             : "working-set allocation failed");
    }
  }
  for (size_t i = 0; i < bufs.size(); ++i) {
    dfree(c, *bufs[i].field);
    *bufs[i].field = fresh[i];
  }
  c->cap = cap;
  c->working_valid = false;
  return CRM_OK;
}

// Grows a list buffer to hold `need` entries (new buffer first, then the old
// one is released).
template <typename T>
crm_status ensure_list(crm_ctx* c, T*& buf, int64_t& cap, int64_t need, int64_t want = -1) {
  if (need <= cap && buf) return CRM_OK;
  const int64_t n = want >= need ? want : (int64_t)std::ceil(c->prm.grow_G * (double)need) + crm::kWave;
  T* nb = nullptr;
  if (!alloc_n(c, nb, n))
    return fail(c, CRM_E_NOMEM, c->noalloc ? "the neighbour lists must grow (a call that may allocate is needed)"
                                           : "neighbour-list allocation failed");
  dfree(c, buf);
  buf = nb;
  cap = n;
  return CRM_OK;
}

// Chunks of the segments [start[g], start[g + 1]) for segment_reduce; device
// arrays from the context's allocator, listed in `owned` when given (freed by
// the caller), else kept for the context's lifetime.
crm_status make_plan(crm_ctx* c, const std::vector<int64_t>& start, crm::SegPlan& plan, std::vector<void*>* owned) {
  const int32_t nseg = (int32_t)start.size() - 1;
  const int64_t ch = crm::reduce_chunk();
  std::vector<int64_t> lo, hi;
  std::vector<int32_t> first((size_t)nseg + 1, 0);
  for (int32_t g = 0; g < nseg; ++g) {
    first[g] = (int32_t)lo.size();
    for (int64_t k = start[g]; k < start[g + 1]; k += ch) {
      lo.push_back(k);
      hi.push_back(std::min(k + ch, start[g + 1]));
    }
  }
  first[nseg] = (int32_t)lo.size();
  const int64_t nc = (int64_t)lo.size();
  int64_t *dlo = nullptr, *dhi = nullptr;
  int32_t* dfirst = nullptr;
  double* dpart = nullptr;
  if (!(alloc_n(c, dlo, nc > 0 ? nc : 1) && alloc_n(c, dhi, nc > 0 ? nc : 1) && alloc_n(c, dfirst, nseg + 1) &&
        alloc_n(c, dpart, 6 * (nc > 0 ? nc : 1))))
    return fail(c, CRM_E_NOMEM, "reduction plan allocation failed");
  if (owned) {
    owned->push_back(dlo);
    owned->push_back(dhi);
    owned->push_back(dfirst);
    owned->push_back(dpart);
  }
  hipStream_t s = c->stream;
  if (nc > 0) {
    HIPCHK(c, hipMemcpyAsync(dlo, lo.data(), sizeof(int64_t) * (size_t)nc, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(dhi, hi.data(), sizeof(int64_t) * (size_t)nc, hipMemcpyHostToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(dfirst, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  plan.nseg = nseg;
  plan.nchunk = nc;
  plan.lo = dlo;
  plan.hi = dhi;
  plan.first = dfirst;
  plan.partial = dpart;
  return CRM_OK;
}

// Writes the chunk plan of the segments [start[g], start[g + 1]) (start:
// nseg + 1 values) into the plan's existing arrays (capacity cap chunks),
// through the context's host plan buffers.
crm_status fill_plan(crm_ctx* c, const int64_t* start, int32_t nseg, crm::SegPlan& plan, int64_t cap) {
  const int64_t ch = crm::reduce_chunk();
  int64_t nc = 0;
  for (int32_t g = 0; g < nseg; ++g)
    for (int64_t k = start[g]; k < start[g + 1]; k += ch) ++nc;
  if (nc > cap) return fail(c, CRM_E_STATE, "force-sum plan exceeds its capacity");
  if ((int64_t)c->plan_lo.size() < nc || (int64_t)c->plan_first.size() < nseg + 1) {
    if (c->noalloc) return fail(c, CRM_E_NOMEM, "the force-sum plan must grow (a call that may allocate is needed)");
    c->plan_lo.resize((size_t)nc);
    c->plan_hi.resize((size_t)nc);
    c->plan_first.resize((size_t)nseg + 1);
  }
  int64_t* lo = c->plan_lo.data();
  int64_t* hi = c->plan_hi.data();
  int32_t* first = c->plan_first.data();
  int64_t q = 0;
  for (int32_t g = 0; g < nseg; ++g) {
    first[g] = (int32_t)q;
    for (int64_t k = start[g]; k < start[g + 1]; k += ch, ++q) {
      lo[q] = k;
      hi[q] = std::min(k + ch, start[g + 1]);
    }
  }
  first[nseg] = (int32_t)q;
  hipStream_t s = c->stream;
  if (nc > 0) {
    HIPCHK(c, hipMemcpyAsync(const_cast<int64_t*>(plan.lo), lo, sizeof(int64_t) * (size_t)nc, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(const_cast<int64_t*>(plan.hi), hi, sizeof(int64_t) * (size_t)nc, hipMemcpyHostToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(const_cast<int32_t*>(plan.first), first, sizeof(int32_t) * (size_t)(nseg + 1),
                           hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  plan.nseg = nseg;
  plan.nchunk = nc;
  return CRM_OK;
}

crm_status read_counts(crm_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->h_counts, c->d_counts, sizeof(uint64_t) * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CRM_OK;
}

// Markers of the bodies that moved since their last placement in the master
// store (all of them after init or a restore): x = X + R l.
// World-axis box around the body's active box grown by ext on every local
// axis, widened by a margin far above FP64 rounding: a superset of the grown
// box used only to skip its exact test.
// The same box as FP32 bounds rounded outwards (a stored FP32 coordinate inside
// alo..ahi lies inside flo..fhi) and as the cell indices a cell-offset
// position inside it can carry (its offset stays within one cell of [0, S),
// so c S lies within 2 S of x - lo).
void set_box_bounds(Body& B, const Grid& g) {
  const double ext = g.ext;
  double mag = 1.0;
  for (int a = 0; a < 3; ++a) mag += std::fabs(B.X[a]) + B.half[a] + ext;
  const double margin = 1e-9 * mag;
  for (int k = 0; k < 3; ++k) {
    double r = 0.0;
    for (int a = 0; a < 3; ++a) r += std::fabs(B.R[3 * k + a]) * (B.half[a] + ext);
    B.alo[k] = B.X[k] - r - margin;
    B.ahi[k] = B.X[k] + r + margin;
    float lo = (float)B.alo[k], hi = (float)B.ahi[k];
    if ((double)lo > B.alo[k]) lo = std::nextafter(lo, -INFINITY);
    if ((double)hi < B.ahi[k]) hi = std::nextafter(hi, INFINITY);
    B.flo[k] = lo;
    B.fhi[k] = hi;
    const double cl = std::floor((B.alo[k] - g.lo[k]) * g.inv) - 2.0;
    const double ch = std::floor((B.ahi[k] - g.lo[k]) * g.inv) + 2.0;
    B.clo[k] = (int32_t)std::max(cl, -2147483647.0);
    B.chi[k] = (int32_t)std::min(ch, 2147483647.0);
  }
}

crm_status place_master_markers(crm_ctx* c) {
  const int64_t* bs = c->h_bstart.data();
  if (c->placed.size() != (size_t)c->nb) {
    c->placed.assign((size_t)c->nb, Body{});
    c->place_all = true;
  }
  for (int b = 0; b < c->nb; ++b) {
    const Body& B = c->h_bodies[b];
    const Body& Q = c->placed[b];
    const bool moved = c->place_all || std::memcmp(B.X, Q.X, sizeof(B.X)) != 0 || std::memcmp(B.R, Q.R, sizeof(B.R)) != 0;
    if (!moved) continue;
    HIPCHK(c, crm::place_markers_master(c->local, bs[b], bs[b + 1], c->n_soil, c->d_bodies, c->grid, c->m_a, c->m_d,
                                        c->m_key,
                                        c->stream));
    c->placed[b] = B;
  }
  c->place_all = false;
  return CRM_OK;
}

// Chunks of the per-body force sums over the processed markers: all markers by
// id when every particle is processed (a fixed plan), else the bodies' ranges
// in the processed list, found on the device and read back.
crm_status update_body_plan(crm_ctx* c, const int32_t* ids) {
  if (c->nb == 0) return CRM_OK;
  if (!ids && c->plan_all) return CRM_OK;
  HIPCHK(c, crm::body_ranges(ids, c->n_proc, c->n_soil, c->d_bstart, c->nb, c->kbase, c->d_branges, c->stream));
  int64_t* r = c->plan_r.data();
  HIPCHK(c, hipMemcpyAsync(r, c->d_branges, sizeof(int64_t) * (size_t)(c->nb + 1), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  crm_status st = fill_plan(c, r, c->nb, c->body_plan, c->plan_cap);
  if (st != CRM_OK) return st;
  c->plan_all = (ids == nullptr);
  return CRM_OK;
}

hipEvent_t prof_begin(crm_ctx* c, int k);
void prof_end(crm_ctx* c, int k, hipEvent_t start);

// The cell grid a rebuild sorts into. With active domains every processed
// particle lies inside the union of the bodies' world boxes (alo..ahi, a
// superset of the boxes grown by the list radius), so the rebuild sorts into
// the window of the domain's grid that covers that union with two cells to
// spare on each side (a stored cell of a cell-offset position is within one
// cell of its position's): the same cells and order, over a few thousand
// cells instead of the whole domain's.
Grid rebuild_grid(const crm_ctx* c, int64_t& cells) {
  Grid w = c->grid;
  cells = c->M;
  if (!c->ad_on) return w;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool any = false;
  for (int b = 0; b < c->nb; ++b) {
    const Body& B = c->h_bodies[b];
    if (!B.has_box) continue;
    any = true;
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], B.alo[k]);
      hi[k] = std::max(hi[k], B.ahi[k]);
    }
  }
  if (!any) return w;
  int64_t m = 1;
  for (int k = 0; k < 3; ++k) {
    const double a = std::floor((lo[k] - w.lo[k]) * w.inv) - 2.0, b = std::floor((hi[k] - w.lo[k]) * w.inv) + 2.0;
    const int32_t c0 = (int32_t)std::max(0.0, std::min(a, (double)(w.gdim[k] - 1)));
    const int32_t c1 = (int32_t)std::max((double)c0, std::min(b, (double)(w.gdim[k] - 1)));
    w.org[k] = c0;
    w.dims[k] = c1 - c0 + 1;
    m *= (int64_t)w.dims[k];
  }
  cells = m;
  return w;
}

// The working set back into the master store: the soil rows of state A (all
// four planes) and the extrapolated velocity and stress of the processed
// markers from the last stage (B), so that the master holds every particle's
// values from the last step it was processed in, whether or not the state was
// read in between.
crm_status scatter_back(crm_ctx* c) {
  hipStream_t s = c->stream;
  HIPCHK(c, crm::scatter_rows(c->A, c->frows, c->n_frows, c->slot_id, c->m_a, c->m_b, c->m_c, c->m_d, c->m_key,
                              c->grid.cell != 0, s));
  HIPCHK(c, crm::scatter_marker_rows(c->B, c->mrows, c->n_mrows, c->slot_id, c->m_b, c->m_c, c->m_d, s));
  return CRM_OK;
}

// Alg. 3 lines for a rebuild step: activity (t > t_delay), count, capacity,
// then PreprocessNeighborList + Algorithm 1 on the processed set.
// The active-domain flags and their per-tile counts from the coarse-cell
// index (same flags as the scan of all N): the index is (re)built when stale
// or when the moved list overflowed; the markers of bodies that moved since
// then join the moved list; the last flags are cleared; the particles listed
// under the coarse cells that the bodies' pre-test cell ranges touch, and
// those on the moved list, are tested.
crm_status activity_by_index(crm_ctx* c, hipStream_t s) {
  const int64_t N = c->n_total;
  const int64_t nw = crm::flags_padded(N) / 4;            // the byte arrays as words
  // markers that would join the moved list now (bodies moved since the index)
  auto pending = [&]() {
    int64_t k = 0;
    for (int b = 0; b < c->nb; ++b) {
      const Body& B = c->h_bodies[b];
      const Body& Q = c->ix_bodies[b];
      if (!c->ix_moving[b] && (std::memcmp(B.X, Q.X, sizeof(B.X)) != 0 || std::memcmp(B.R, Q.R, sizeof(B.R)) != 0))
        k += c->h_bstart[b + 1] - c->h_bstart[b];
    }
    return k;
  };
  // h_counts[6]: the moved list's length after the last rebuild's additions
  if (!c->ix_valid || (int64_t)c->h_counts[6] + pending() > c->mcap) {
    HIPCHK(c, crm::ix_build(c->m_a, c->m_d, N, c->grid, c->ix_start, c->ix_fill, c->ix_scan, c->ix_ids, s));
    HIPCHK(c, crm::fill_u32(reinterpret_cast<uint32_t*>(c->moved), 0u, nw, s));
    HIPCHK(c, crm::fill_u32(reinterpret_cast<uint32_t*>(c->d_counts + 6), 0u, 2, s));
    c->h_counts[6] = 0;
    c->ix_bodies = c->h_bodies;
    c->ix_moving.assign((size_t)c->nb, 0);
    c->ix_valid = true;
    c->flags_valid = false;
  }
  for (int b = 0; b < c->nb; ++b) {
    const Body& B = c->h_bodies[b];
    const Body& Q = c->ix_bodies[b];
    if (c->ix_moving[b] || (std::memcmp(B.X, Q.X, sizeof(B.X)) == 0 && std::memcmp(B.R, Q.R, sizeof(B.R)) == 0))
      continue;
    const int64_t k0 = c->h_bstart[b], k1 = c->h_bstart[b + 1];
    HIPCHK(c, crm::moved_add(nullptr, nullptr, k1 - k0, nullptr, c->n_soil + k0, c->moved, c->mlist, c->d_counts + 6,
                             c->mcap, s));
    c->ix_moving[b] = 1;
  }
  if (c->flags_valid)
    HIPCHK(c, crm::flags_clear(c->proc_ids, c->d_counts, N, c->flags, s));
  else
    HIPCHK(c, crm::fill_u32(reinterpret_cast<uint32_t*>(c->flags), 0u, nw, s));
  HIPCHK(c, crm::fill_u32(c->ctmp, 0u, crm::flag_tiles(N), s));
  // the coarse cells that the bodies' pre-test cell ranges touch
  c->h_visit.clear();
  const int32_t kc = crm::coarse_size();
  for (const Body& B : c->h_bodies) {
    if (!B.has_box) continue;
    int32_t lo[3], hi[3];
    bool empty = false;
    for (int k = 0; k < 3; ++k) {
      const int32_t a = std::max(B.clo[k], 0), z = std::min(B.chi[k], c->grid.gdim[k] - 1);
      if (a > z) empty = true;
      lo[k] = a / kc;
      hi[k] = z / kc;
    }
    if (empty) {   // a range beyond the grid: its edge cells hold the particles outside
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(std::max(B.clo[k], 0), c->grid.gdim[k] - 1) / kc;
        hi[k] = std::min(std::max(B.chi[k], 0), c->grid.gdim[k] - 1) / kc;
      }
    }
    for (int32_t z = lo[2]; z <= hi[2]; ++z)
      for (int32_t y = lo[1]; y <= hi[1]; ++y)
        for (int32_t x = lo[0]; x <= hi[0]; ++x)
          c->h_visit.push_back(((uint32_t)z * (uint32_t)c->ix_cd[1] + (uint32_t)y) * (uint32_t)c->ix_cd[0] +
                               (uint32_t)x);
  }
  std::sort(c->h_visit.begin(), c->h_visit.end());
  c->h_visit.erase(std::unique(c->h_visit.begin(), c->h_visit.end()), c->h_visit.end());
  const int64_t nv = (int64_t)c->h_visit.size();
  if (nv > 0) {
    // the last upload from the pinned list has completed: every rebuild reads
    // its counts back (a stream synchronisation) after this copy
    std::memcpy(c->h_visit_pin, c->h_visit.data(), sizeof(uint32_t) * (size_t)nv);
    HIPCHK(c, hipMemcpyAsync(c->ix_visit, c->h_visit_pin, sizeof(uint32_t) * (size_t)nv, hipMemcpyHostToDevice, s));
  }
  HIPCHK(c, crm::ix_flags(c->ix_visit, nv, c->ix_start, c->ix_ids, c->moved, c->mlist, c->d_counts + 6, c->mcap,
                          c->m_key, c->m_a, c->m_d, c->d_bodies, c->nb, c->grid, c->flags, c->ctmp, s));
  return CRM_OK;
}

crm_status rebuild(crm_ctx* c) {
  hipStream_t s = c->stream;
  const crm_params& P = c->prm;
  if (c->working_valid) {
    crm_status st0 = scatter_back(c);
    if (st0 != CRM_OK) return st0;
  }
  // from here until the rebuild completes the master store is the state: a
  // rebuild that fails (e.g. an allocation) leaves the state as it was, and
  // the next step starts the rebuild again
  c->working_valid = false;
  if (c->recording) {
    // the state every later step of this segment follows from (reverse mode)
    const int64_t k = (int64_t)c->rec_seg.size();
    if (k >= c->rec_snap_cap) return fail(c, CRM_E_STATE, "more list rebuilds than the record expected");
    const size_t n = (size_t)c->n_total;
    float4* dst = c->rec_snap + (size_t)k * 4 * n;
    const float4* src[4] = {c->m_a, c->m_b, c->m_c, c->m_d};
    for (int q = 0; q < 4; ++q)
      HIPCHK(c, hipMemcpyAsync(dst + q * n, src[q], sizeof(float4) * n, hipMemcpyDeviceToDevice, s));
    c->rec_seg.push_back(c->step - c->rec_step0);
  }
  {
    crm_status st0 = place_master_markers(c);
    if (st0 != CRM_OK) return st0;
  }
  const double t = (double)c->step * P.dt;
  c->ad_on = P.active_domains && t > P.t_delay;
  int64_t n_proc = c->n_total;
  // the index while the integrated rows fill at most half the moved list
  // (more: the test of all N costs less than the index's upkeep)
  c->ix_used = c->ad_on && c->ix_on && 2 * c->n_frows <= c->mcap;
  if (c->ix_used) {
    hipEvent_t ea = prof_begin(c, 7);
    crm_status st = activity_by_index(c, s);
    if (st != CRM_OK) return st;
    prof_end(c, 7, ea);
    HIPCHK(c, crm::compact_counted(c->flags, c->n_total, c->proc_ids, c->d_counts, c->ctmp, s));
    st = read_counts(c);
    if (st != CRM_OK) return st;
    n_proc = (int64_t)c->h_counts[0];
    c->flags_valid = true;
  } else if (c->ad_on) {
    hipEvent_t ea = prof_begin(c, 7);
    crm::ActUnion un;
    for (int k = 0; k < 3; ++k) {
      un.flo[k] = INFINITY;
      un.fhi[k] = -INFINITY;
      un.clo[k] = INT32_MAX;
      un.chi[k] = INT32_MIN;
    }
    for (const Body& B : c->h_bodies) {
      if (!B.has_box) continue;
      for (int k = 0; k < 3; ++k) {
        un.flo[k] = std::min(un.flo[k], B.flo[k]);
        un.fhi[k] = std::max(un.fhi[k], B.fhi[k]);
        un.clo[k] = std::min(un.clo[k], B.clo[k]);
        un.chi[k] = std::max(un.chi[k], B.chi[k]);
      }
    }
    HIPCHK(c, crm::activity_count(c->m_a, c->m_d, c->m_key, c->n_total, c->d_bodies, c->nb, un, c->grid, c->flags,
                                  c->ctmp, s));
    prof_end(c, 7, ea);
    HIPCHK(c, crm::compact_counted(c->flags, c->n_total, c->proc_ids, c->d_counts, c->ctmp, s));
    crm_status st = read_counts(c);
    if (st != CRM_OK) return st;
    n_proc = (int64_t)c->h_counts[0];
    c->ix_valid = false;      // the rows integrated from here on are not tracked
    c->flags_valid = false;
  } else {
    // every particle processed (and the soil integrated): the index is stale
    c->ix_valid = false;
    c->flags_valid = false;
  }
  // capacity policy (Sec. 4.2 item 3)
  int64_t ncap = crm_capacity_next(c->cap, n_proc, c->step, P.grow_G, P.shrink_S, P.shrink_interval);
  // a call that must not allocate keeps a larger working set (the results do
  // not depend on the capacity); the shrink waits for a call that may allocate
  if (c->noalloc && c->A.a && ncap < c->cap && n_proc <= c->cap) ncap = c->cap;
  if (ncap != c->cap || !c->A.a) {
    crm_status st = realloc_working(c, ncap);
    if (st != CRM_OK) return st;
  }
  c->n_proc = n_proc;
  const int32_t* ids = c->ad_on ? c->proc_ids : nullptr;
  const uint8_t* flg = c->ad_on ? c->flags : nullptr;
  int64_t Mw = c->M;
  const Grid g = rebuild_grid(c, Mw);
  c->wgrid = g;
  c->Mw = Mw;
  Phys pw = c->phys;
  for (int k = 0; k < 3; ++k) pw.gdim[k] = g.dims[k];
  HIPCHK(c, crm::fill_u32(c->cell_cnt, 0u, Mw, s));
  HIPCHK(c, crm::hash_count(ids, n_proc, c->m_a, c->m_d, g, c->key, c->rank, c->cell_cnt, s));
  HIPCHK(c, crm::scan_u32_to_u32(c->cell_cnt, c->cell_start, Mw, c->cell_tmp, s));
  HIPCHK(c, crm::place_sorted(c->key, c->rank, c->cell_start, n_proc, ids, c->m_a, c->m_d, c->tmp, c->tmpx,
                              c->grid.cell != 0, s));
  HIPCHK(c, crm::gather_sorted(c->tmp, c->tmpx, c->key, ids, c->cell_start, n_proc, c->n_soil, flg, c->m_a, c->m_b, c->m_c,
                               c->m_d, c->A, c->B, c->pos4, c->cpos, c->slot_id, c->slot_k, c->skey,
                               c->grid.cell != 0, s));
  HIPCHK(c, crm::compact_kind(c->pos4, n_proc, crm::kSoilActive, c->frows, c->d_counts + 1, c->ctmp, s));
  HIPCHK(c, crm::compact_kind(c->pos4, n_proc, crm::kMarker, c->mrows, c->d_counts + 2, c->ctmp, s));
  // the row lists hold at most this many rows (their counts are on the device):
  // the soil and marker passes and scans run over these bounds, not n_proc
  const int64_t rf = std::min(n_proc, c->n_soil), rm = std::min(n_proc, c->n_mark);
  // the rows integrated until the next rebuild leave their place in the index
  if (c->ix_used)
    HIPCHK(c, crm::moved_add(c->frows, c->d_counts + 1, rf, c->slot_id, 0, c->moved, c->mlist, c->d_counts + 6,
                             c->mcap, s));
  HIPCHK(c, crm::tile_tables(c->frows, rf, c->d_counts + 1, c->skey, c->cell_start, pw, c->tabs, s));
  HIPCHK(c, crm::nbr_count_soil(c->frows, rf, c->d_counts + 1, c->pos4, c->cpos, c->skey, c->cell_start, g,
                                c->tabs, c->cnt_f, c->stash_f, s));
  HIPCHK(c, crm::scan_u32_to_u64(c->cnt_f, c->off_f, rf, c->wtmp, s));
  HIPCHK(c, crm::nbr_count(c->mrows, rm, c->d_counts + 2, c->pos4, c->cpos, c->skey, c->cell_start, g,
                           true, c->cnt_m, c->stash_m, s));
  HIPCHK(c, crm::scan_u32_to_u64(c->cnt_m, c->off_m, rm, c->wtmp, s));
  HIPCHK(c, crm::copy2_u64(c->d_counts + 3, c->off_f + rf, c->off_m + rm, s));
  HIPCHK(c, crm::compact_nonzero(c->cnt_m, rm, c->near, c->d_counts + 5, c->ctmp, s));
  crm_status st = read_counts(c);
  if (st != CRM_OK) return st;
  c->n_frows = (int64_t)c->h_counts[1];
  c->n_mrows = (int64_t)c->h_counts[2];
  c->n_near = (int64_t)c->h_counts[5];
  HIPCHK(c, crm::near_rows(c->mrows, c->near, c->n_near, c->off_m, c->nrow, s));
  // the force entries of markers without soil neighbours stay zero until the
  // next rebuild (the BCE passes skip them)
  HIPCHK(c, crm::fill_u32(reinterpret_cast<uint32_t*>(c->contrib), 0u, 12 * c->n_mrows, s));
  const int64_t ef = (int64_t)c->h_counts[3], em = (int64_t)c->h_counts[4];
  st = ensure_list(c, c->nbr_f, c->nbr_f_cap, ef);
  if (st != CRM_OK) return st;
  st = ensure_list(c, c->tix_f, c->tix_f_cap, ef, c->nbr_f_cap);
  if (st != CRM_OK) return st;
  st = ensure_list(c, c->nbr_m, c->nbr_m_cap, em);
  if (st != CRM_OK) return st;
  c->ent_f = ef;
  c->ent_m = em;
  // the slots of the blocks the stages read from their tiles are left out
  // (written on demand by complete_lists)
  const uint32_t skip = c->full_lists ? 0u : crm::tile_records(c->tile_cfg, c->grid.cell != 0);
  HIPCHK(c, crm::nbr_fill_soil(c->frows, c->n_frows, c->pos4, c->cpos, c->skey, c->cell_start, g, c->cnt_f,
                               c->stash_f, c->off_f, c->nbr_f, c->tabs, c->tix_f, skip, s));
  c->nbr_skip = skip;
  HIPCHK(c, crm::nbr_fill(c->mrows, c->n_mrows, c->pos4, c->cpos, c->skey, c->cell_start, g, true,
                          c->cnt_m, c->stash_m, c->off_m, c->nbr_m, s));
  // every marker row of the new working set placed once (rows that lost or
  // gained soil neighbours, values gathered from the master store)
  HIPCHK(c, crm::place_markers_working(c->mrows, c->n_mrows, c->cnt_m, c->slot_id, c->n_soil, c->local, c->d_bodies,
                                       c->grid, c->phys, c->A, c->B, true, s));
  // per-body ranges of the processed markers for the force sums
  c->kbase = c->n_proc - c->n_mrows;
  st = update_body_plan(c, ids);
  if (st != CRM_OK) return st;
  // the stage kernels' block order for these rows: chunked along x where a
  // plane of rows of cells (the reuse distance of a record in cell order)
  // holds more than ~2 MB of stage records, a good part of an XCD's 4 MB L2;
  // cell order otherwise, or when the window's order table exceeds the one
  // sized at crm_init. (Measured: 64 bins of 8k-250k soil particles laid
  // along x, 5.7 MB per plane, a step 3.37 -> 2.98 ms; the single-wheel bin,
  // 0.8 MB per plane, stage 2 5 % slower when chunked.)
  c->phys.bperm = nullptr;
  const double plane_bytes = 52.0 * (double)c->n_frows / (double)std::max(1, g.dims[2]);
  if (c->ord_cap > 0 && c->n_frows > 0 && plane_bytes > 2.0e6 && crm::block_order_size(g) <= c->ord_cap) {
    HIPCHK(c, crm::block_order(c->frows, c->skey, c->n_frows, g, c->ord_cnt, c->ord_first, c->ord_base, c->ord_scan,
                               c->bperm, s));
    c->phys.bperm = c->bperm;
  }
  c->working_valid = true;
  c->force_rebuild = false;
  c->rebuilds += 1;
  c->last_rebuild = c->step;
  if (c->prm.skin > 0.0) {
    HIPCHK(c, crm::fill_u32(c->d_disp, 0u, 1, s));
    c->disp_pending = false;
  }
  return CRM_OK;
}

// Writes the slots the last rebuild left out of nbr_f (for the reverse sweep,
// the exported lists and a change of tile configuration).
crm_status complete_lists(crm_ctx* c) {
  if (!c->working_valid || c->nbr_skip == 0) return CRM_OK;
  HIPCHK(c, crm::nbr_slots(c->n_frows, c->off_f, c->tabs, c->tix_f, c->nbr_f, c->nbr_skip, c->stream));
  c->nbr_skip = 0;
  return CRM_OK;
}

hipEvent_t prof_event(crm_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// Records a start event for kernel class k when it is profiled; returns it.
hipEvent_t prof_begin(crm_ctx* c, int k) {
  if (!c->prof || !((c->prof_mask >> k) & 1u)) return nullptr;
  hipEvent_t e = prof_event(c);
  if (e) (void)hipEventRecord(e, c->stream);
  return e;
}

void prof_end(crm_ctx* c, int k, hipEvent_t start) {
  if (!c->prof || !start) return;
  hipEvent_t e = prof_event(c);
  if (!e) return;
  (void)hipEventRecord(e, c->stream);
  c->prof_marks.push_back({k, {start, e}});
}

// Where a taped step keeps y_n and y_mid (with the markers' extrapolated
// values of each stage) and the tapes of its two stages.
struct StepRecord {
  Planes yn, ym;
  crm::StageTape t1, t2;
};

crm_status copy_planes(crm_ctx* c, CPlanes src, Planes dst, int64_t n, hipStream_t s) {
  const size_t b = sizeof(float4) * (size_t)n;
  if (n <= 0) return CRM_OK;
  HIPCHK(c, hipMemcpyAsync(dst.a, src.a, b, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(dst.b, src.b, b, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(dst.c, src.c, b, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(dst.d, src.d, b, hipMemcpyDeviceToDevice, s));
  return CRM_OK;
}

// The kernels of one step after the (optional) rebuild, on stream s, in two
// parts: up to the body sums (marker placement, BCE, stage 1, BCE with the
// forces, their reduction into the mapped host buffer), then stage 2, which
// the sums do not depend on. Between the two, a direct launch records fpin_ev,
// so that crm_get_forces returns while stage 2 still runs and the caller's
// next body state is computed and enqueued meanwhile.
crm_status launch_head(crm_ctx* c, hipStream_t s, bool prof, const StepRecord* rec) {
  const crm::StageTape* tape1 = rec ? &rec->t1 : nullptr;
  const Phys& P = c->phys;
  hipEvent_t e = prof ? prof_begin(c, 1) : nullptr;
  HIPCHK(c, crm::place_markers_working(c->mrows, c->n_mrows, c->cnt_m, c->slot_id, c->n_soil, c->local,
                                       c->d_bodies, c->grid, P, c->A, c->B, false, s));
  if (prof) prof_end(c, 1, e);
  // stage 1 at y_n
  if (prof) e = prof_begin(c, 2);
  HIPCHK(c, crm::bce(c->A, c->nrow, c->n_near, c->nbr_m, c->d_bodies, c->slot_k, c->kbase, P, nullptr, s));
  if (prof) prof_end(c, 2, e);
  if (rec) {
    crm_status st = copy_planes(c, c->A, rec->yn, c->n_proc, s);
    if (st != CRM_OK) return st;
  }
  if (prof) e = prof_begin(c, 3);
  HIPCHK(c, crm::fluid_stage1(c->A, c->B, c->frows, c->n_frows, c->off_f, c->nbr_f, P, tape1, c->tabs, c->tix_f,
                              c->tile_cfg, s));
  if (prof) prof_end(c, 3, e);
  // the markers at y_mid and the body forces from this evaluation
  if (prof) e = prof_begin(c, 4);
  HIPCHK(c, crm::bce(c->B, c->nrow, c->n_near, c->nbr_m, c->d_bodies, c->slot_k, c->kbase, P, c->contrib, s));
  if (prof) prof_end(c, 4, e);
  if (rec) {
    crm_status st = copy_planes(c, c->B, rec->ym, c->n_proc, s);
    if (st != CRM_OK) return st;
  }
  if (prof) e = prof_begin(c, 6);
  HIPCHK(c, crm::segment_reduce(c->contrib, c->body_plan, c->d_fmap, s, c->d_fseq));
  if (prof) prof_end(c, 6, e);
  return CRM_OK;
}

// Stage 2 at y_mid.
crm_status launch_tail(crm_ctx* c, hipStream_t s, bool prof, const StepRecord* rec) {
  const crm::StageTape* tape2 = rec ? &rec->t2 : nullptr;
  hipEvent_t e = prof ? prof_begin(c, 5) : nullptr;
  HIPCHK(c, crm::fluid_stage2(c->B, c->A, c->frows, c->n_frows, c->off_f, c->nbr_f, c->phys, tape2, c->tabs,
                              c->tix_f, c->tile_cfg, s));
  if (prof) prof_end(c, 5, e);
  return CRM_OK;
}

// Notes that the body sums just enqueued on the context's stream (their
// reduction moves every body's counter by one) are those of the step in
// progress (c->step before its increment). Every executed reduction of the
// step kernels is enqueued through here, so the counters equal fseq once the
// last one has written its sums.
crm_status mark_forces(crm_ctx* c) {
  c->fseq += 1;
  c->fpin_step = c->step + 1;
  return CRM_OK;
}

crm_status launch_step(crm_ctx* c, hipStream_t s, bool prof, const StepRecord* rec = nullptr) {
  crm_status st = launch_head(c, s, prof, rec);
  if (st == CRM_OK && s == c->stream && c->nb > 0) st = mark_forces(c);
  if (st == CRM_OK) st = launch_tail(c, s, prof, rec);
  return st;
}

void drop_graph(crm_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->gexec2) (void)hipGraphExecDestroy(c->gexec2);
  if (c->graph2) (void)hipGraphDestroy(c->graph2);
  c->gexec = c->gexec2 = nullptr;
  c->graph = c->graph2 = nullptr;
  c->graph_key.clear();
}

// One part of a step captured on the capture stream and instantiated.
crm_status capture_part(crm_ctx* c, bool head, hipGraph_t* g, hipGraphExec_t* x) {
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  crm_status st = head ? launch_head(c, c->cap_stream, false, nullptr) : launch_tail(c, c->cap_stream, false, nullptr);
  hipGraph_t gg = nullptr;
  hipError_t ee = hipStreamEndCapture(c->cap_stream, &gg);
  if (st != CRM_OK) {
    if (gg) (void)hipGraphDestroy(gg);
    return st;
  }
  if (ee != hipSuccess) return fail(c, CRM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
  *g = gg;
  HIPCHK(c, hipGraphInstantiate(x, gg, nullptr, nullptr, 0));
  return CRM_OK;
}

// Everything the captured kernels bake in: buffers and row counts.
std::vector<const void*> graph_key(const crm_ctx* c) {
  return {c->A.a, c->B.a, c->frows, c->mrows, c->near, c->nrow, c->off_f, c->off_m, c->nbr_f, c->nbr_m, c->tix_f, c->slot_id,
          c->contrib, (const void*)(intptr_t)c->n_frows, (const void*)(intptr_t)c->n_mrows,
          (const void*)(intptr_t)c->n_near,
          (const void*)(intptr_t)c->tile_cfg, (const void*)(intptr_t)c->body_plan.nchunk, c->phys.bperm,
          (const void*)(intptr_t)c->kbase};
}

crm_status step_graph(crm_ctx* c) {
  std::vector<const void*> key = graph_key(c);
  if (!c->gexec || !c->gexec2 || key != c->graph_key) {
    drop_graph(c);
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    crm_status st = capture_part(c, true, &c->graph, &c->gexec);
    if (st == CRM_OK) st = capture_part(c, false, &c->graph2, &c->gexec2);
    if (st != CRM_OK) {
      drop_graph(c);
      return st;
    }
    c->graph_key = key;
  }
  HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  if (c->nb > 0) {
    crm_status st = mark_forces(c);
    if (st != CRM_OK) return st;
  }
  HIPCHK(c, hipGraphLaunch(c->gexec2, c->stream));
  return CRM_OK;
}

// Squared displacement read back after the last step exceeds (skin / 2)^2.
bool moved_beyond_half_skin(crm_ctx* c) {
  if (!c->disp_pending) return false;
  (void)hipEventSynchronize(c->disp_ev);
  float d2;
  std::memcpy(&d2, c->h_disp, 4);
  const double half = 0.5 * c->prm.skin;
  return (double)d2 > half * half;
}

bool rebuild_due(crm_ctx* c) {
  if (c->force_rebuild || !c->working_valid) return true;
  if (c->prm.skin <= 0.0) return c->step % (int64_t)c->prm.ps_freq == 0;
  return c->step - c->last_rebuild >= (int64_t)c->prm.ps_freq || moved_beyond_half_skin(c);
}

// Verlet lists: the largest displacement since the rebuild, read back
// asynchronously for the next step's decision.
crm_status track_displacement(crm_ctx* c) {
  if (c->prm.skin <= 0.0) return CRM_OK;
  hipStream_t s = c->stream;
  HIPCHK(c, crm::max_disp(c->A, c->pos4, c->cpos, c->n_proc, c->grid.cell != 0, c->phys.Sf, c->d_disp, s));
  HIPCHK(c, hipMemcpyAsync(c->h_disp, c->d_disp, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipEventRecord(c->disp_ev, s));
  c->disp_pending = true;
  return CRM_OK;
}

// The body states the step just placed its markers with (sized at crm_init:
// no allocation here).
void note_placement(crm_ctx* c) {
  std::copy(c->h_bodies.begin(), c->h_bodies.begin() + c->nb, c->wplaced.begin());
  c->wplaced_ok = true;
}

crm_status one_step(crm_ctx* c, const StepRecord* rec = nullptr) {
  if (rebuild_due(c)) {
    hipEvent_t e = prof_begin(c, 0);
    crm_status st = rebuild(c);
    if (st != CRM_OK) return st;
    prof_end(c, 0, e);
  }
  crm_status st = rec ? launch_step(c, c->stream, false, rec)
                      : (c->use_graph && !c->prof) ? step_graph(c) : launch_step(c, c->stream, c->prof);
  if (st != CRM_OK) return st;
  note_placement(c);
  st = track_displacement(c);
  if (st != CRM_OK) return st;
  c->step += 1;
  c->stepped = true;
  return CRM_OK;
}

void release(crm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  std::vector<Buf> all = c->owned;
  for (auto& b : all) dfree(c, b.p);
  if (c->h_counts) (void)hipHostFree(c->h_counts);
  if (c->h_disp) (void)hipHostFree(c->h_disp);
  if (c->h_bpin) (void)hipHostFree(c->h_bpin);
  if (c->h_fpin) (void)hipHostFree(c->h_fpin);
  if (c->h_visit_pin) (void)hipHostFree(c->h_visit_pin);
  if (c->bpin_ev) (void)hipEventDestroy(c->bpin_ev);
  if (c->fpin_ev) (void)hipEventDestroy(c->fpin_ev);
  if (c->disp_ev) (void)hipEventDestroy(c->disp_ev);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

// Waits for ev by polling (a co-simulation exchange waits for every step:
// polling avoids the wake-up latency of a blocking wait).
hipError_t poll_event(hipEvent_t ev) {
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e != hipErrorNotReady) return e;
  }
}

crm_status usable(crm_ctx* c) {
  if (!c) return fail(nullptr, CRM_E_INVALID, "ctx is NULL");
  if (c->poisoned) return fail(c, CRM_E_STATE, "context is poisoned by an earlier device error: " + c->err);
  return CRM_OK;
}

// Sub-ranges of the static scratch array for the transient buffers of a step:
// compaction block counts, the cell scan's and the list scans' tile totals and
// the body-force chunk sums. Returns the bytes needed (0 on overflow).
struct ScratchLayout {
  uint32_t* ctmp = nullptr;
  uint32_t* cell_tmp = nullptr;
  uint64_t* wtmp = nullptr;
  double* partial = nullptr;
  size_t bytes = 0;
};

ScratchLayout scratch_layout(const crm_ctx* c) {
  ScratchLayout L;
  auto take = [&](size_t b) {
    const size_t at = L.bytes;
    L.bytes += (b + 255) & ~size_t(255);
    return at;
  };
  const size_t o_ctmp = take(sizeof(uint32_t) * crm::compact_tmp_elems(c->n_total));
  const size_t o_cell = take(sizeof(uint32_t) * crm::scan_tmp_elems(c->M));
  const size_t o_wtmp = take(sizeof(uint64_t) * crm::scan_tmp_elems(c->cap));
  const size_t o_part = take(sizeof(double) * 6 * (size_t)(c->plan_cap > 0 ? c->plan_cap : 1));
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  L.ctmp = reinterpret_cast<uint32_t*>(base + o_ctmp);
  L.cell_tmp = reinterpret_cast<uint32_t*>(base + o_cell);
  L.wtmp = reinterpret_cast<uint64_t*>(base + o_wtmp);
  L.partial = reinterpret_cast<double*>(base + o_part);
  return L;
}

// For the duration of a call that must not allocate: the context's transient
// buffers point into the static scratch, and every allocation fails.
struct NoAllocScope {
  crm_ctx* c;
  uint32_t *ctmp, *cell_tmp;
  uint64_t* wtmp;
  double* partial;
  NoAllocScope(crm_ctx* ctx, const ScratchLayout& L)
      : c(ctx), ctmp(ctx->ctmp), cell_tmp(ctx->cell_tmp), wtmp(ctx->wtmp), partial(ctx->body_plan.partial) {
    c->ctmp = L.ctmp;
    c->cell_tmp = L.cell_tmp;
    c->wtmp = L.wtmp;
    c->body_plan.partial = L.partial;
    c->noalloc = true;
  }
  ~NoAllocScope() {
    c->ctmp = ctmp;
    c->cell_tmp = cell_tmp;
    c->wtmp = wtmp;
    c->body_plan.partial = partial;
    c->noalloc = false;
  }
};

}  // namespace

extern "C" {

int64_t crm_capacity_next(int64_t cap, int64_t n, int64_t step, double G, double S, int64_t S_I) {
  if (n > cap) return (int64_t)std::ceil(G * (double)n);
  if (S_I > 0 && step % S_I == 0 && cap > 0 && (double)n / (double)cap < S) return n;
  return cap;
}

const char* crm_last_error(const crm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

crm_status crm_init(const crm_params* params, int64_t n_soil, const double* pos, const float* vel,
                    const float* sigma, const float* rho, int32_t n_bodies, const crm_body_desc* bodies,
                    crm_alloc_fn alloc, crm_free_fn free_fn, void* alloc_user, void* hip_stream, crm_ctx** out) {
  if (!out) return fail(nullptr, CRM_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string msg = check_params(params);
  if (!msg.empty()) return fail(nullptr, CRM_E_INVALID, msg);
  if (n_soil < 0) return fail(nullptr, CRM_E_INVALID, "n_soil must be >= 0");
  if (n_soil > 0 && !pos) return fail(nullptr, CRM_E_INVALID, "pos is NULL");
  if (n_bodies < 0 || n_bodies > crm::kMaxBodies) return fail(nullptr, CRM_E_INVALID, "n_bodies out of range");
  if (n_bodies > 0 && !bodies) return fail(nullptr, CRM_E_INVALID, "bodies is NULL");
  if ((alloc == nullptr) != (free_fn == nullptr)) return fail(nullptr, CRM_E_INVALID, "alloc and free must both be set");
  int64_t nm = 0;
  for (int b = 0; b < n_bodies; ++b) {
    if (bodies[b].n_markers < 0) return fail(nullptr, CRM_E_INVALID, "n_markers must be >= 0");
    if (bodies[b].n_markers > 0 && !bodies[b].marker_local) return fail(nullptr, CRM_E_INVALID, "marker_local is NULL");
    for (int a = 0; a < 3; ++a)
      if (!(std::isfinite(bodies[b].active_half[a]) && bodies[b].active_half[a] >= 0.0))
        return fail(nullptr, CRM_E_INVALID, "active_half must be finite and >= 0");
    nm += bodies[b].n_markers;
  }
  const int64_t n_total = n_soil + nm;
  if (n_total < 1) return fail(nullptr, CRM_E_INVALID, "no particles");
  if (n_total > (int64_t)0x7fffffff - 1) return fail(nullptr, CRM_E_UNSUPPORTED, "more than 2^31 - 2 particles");
  for (int64_t i = 0; i < 3 * n_soil; ++i)
    if (!std::isfinite(pos[i])) return fail(nullptr, CRM_E_INVALID, "non-finite position");
  Grid g{};
  // list radius and cell size: 2h, or 2h + skin for Verlet lists
  const double radius = 2.0 * params->h + params->skin;
  g.inv = 1.0 / radius;
  g.R2 = radius * radius;
  g.ext = radius;
  g.S = radius;
  g.Sf = (float)radius;
  g.R2lo = std::nextafter((float)(g.R2 * (1.0 - 0x1p-14)), 0.0f);
  g.R2hi = std::nextafter((float)(g.R2 * (1.0 + 0x1p-14)), INFINITY);
  g.cell = params->pos_mode == CRM_POS_CELL_OFFSET ? 1 : 0;
  int64_t M = 1;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = params->domain_lo[a];
    double d = std::floor((params->domain_hi[a] - params->domain_lo[a]) * g.inv) + 1.0;
    if (!(d >= 1.0 && d < 2.0e9)) return fail(nullptr, CRM_E_UNSUPPORTED, "cell grid too large");
    g.dims[a] = (int32_t)d;
    g.gdim[a] = g.dims[a];
    g.org[a] = 0;
    M *= (int64_t)d;
  }
  if (M > (int64_t)0xfffffffe) return fail(nullptr, CRM_E_UNSUPPORTED, "more than 2^32 - 2 cells");
  if (g.cell && (g.dims[1] > 32767 || g.dims[2] > 32767))
    return fail(nullptr, CRM_E_UNSUPPORTED, "cell-offset positions need fewer than 32768 cells along y and z");
  if (n_total > ((int64_t)1 << 28)) return fail(nullptr, CRM_E_UNSUPPORTED, "more than 2^28 particles");

  crm_ctx* c = new crm_ctx();
  c->prm = *params;
  c->stream = (hipStream_t)hip_stream;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = alloc_user;
  c->n_soil = n_soil;
  c->n_mark = nm;
  c->n_total = n_total;
  c->nb = n_bodies;
  c->grid = g;
  c->M = M;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, CRM_E_DEVICE, "no HIP device");
  }
  {
    const hipError_t e = crm::scratch_address(c->device, &c->scratch);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, CRM_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    }
  }
  c->placed.assign((size_t)n_bodies, Body{});
  c->wplaced.assign((size_t)n_bodies, Body{});

  // physical constants (Sec. 2.1, 2.2)
  const crm_params& P = *params;
  const double G = P.E / (2.0 * (1.0 + P.nu));
  const double K = P.E / (3.0 * (1.0 - 2.0 * P.nu));
  const double cs = std::sqrt(K / P.rho0);
  const double m = P.rho0 * P.dx * P.dx * P.dx;
  const double pi = 3.14159265358979323846;
  Phys& ph = c->phys;
  ph.inv_h = (float)(1.0 / P.h);
  const double h2 = P.h * P.h, h3 = h2 * P.h;
  ph.kern = (int32_t)P.kernel;
  if (P.kernel == CRM_KERNEL_WENDLAND) {
    const double a = 21.0 / (16.0 * pi * h3);
    ph.kw = (float)a;
    ph.kf = (float)(5.0 * a / h2);
    ph.kg = (float)(7.5 * a / (h2 * h2));
  } else {
    ph.kw = (float)(1.0 / (pi * h3));
    ph.kf = (float)(1.0 / (pi * h3 * h2));
    ph.kg = (float)(1.0 / (pi * h3 * h2 * h2));
  }
  ph.h = (float)P.h;
  ph.dt = (float)P.dt;
  ph.half_dt = (float)(0.5 * P.dt);
  ph.gx = (float)P.gravity[0];
  ph.gy = (float)P.gravity[1];
  ph.gz = (float)P.gravity[2];
  ph.m = (float)m;
  ph.rho0 = (float)P.rho0;
  ph.two_G = (float)(2.0 * G);
  ph.iso = (float)(P.bulk_coeff * K - 2.0 * G / 3.0);
  ph.av_coef = (float)(P.av_gamma * P.h * cs * m);
  ph.xi2 = (float)((P.av_xi_over_h * P.h) * (P.av_xi_over_h * P.h));
  ph.av_mode = (int32_t)P.av_mode;
  ph.G = (float)G;
  ph.bulk = (float)P.bulk_coeff;
  ph.inv_2K = (float)(0.5 / K);
  ph.mu_s = (float)P.mu_s;
  ph.mu_2 = (float)P.mu_2;
  ph.I0 = (float)P.I0;
  ph.grain_d = (float)P.grain_d;
  ph.cohesion = (float)P.cohesion;
  ph.p_cri = (float)(-P.cohesion / P.mu_s);
  ph.inv_Gdt = (float)(1.0 / (G * P.dt));
  ph.cell = g.cell;
  ph.Sf = (float)g.S;
  ph.S = g.S;
  ph.invS = g.inv;
  for (int q = 0; q < 3; ++q) {
    ph.lo[q] = g.lo[q];
    ph.gdim[q] = g.dims[q];
  }

  // host staging of the master planes
  std::vector<float4> ha((size_t)n_total), hb((size_t)n_total), hc((size_t)n_total), hd((size_t)n_total);
  std::vector<float4> hl((size_t)(nm > 0 ? nm : 1));
  for (int64_t i = 0; i < n_soil; ++i) {
    float r0 = rho ? rho[i] : (float)P.rho0;
    ha[i] = make_float4(0.f, 0.f, 0.f, r0);
    float v[3] = {0.f, 0.f, 0.f}, sg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (vel)
      for (int a = 0; a < 3; ++a) v[a] = vel[3 * i + a];
    if (sigma)
      for (int a = 0; a < 6; ++a) sg[a] = sigma[6 * i + a];
    uint32_t aux = crm::kSoilActive;
    float auxf;
    std::memcpy(&auxf, &aux, 4);
    hb[i] = make_float4(v[0], v[1], v[2], auxf);
    hc[i] = make_float4(sg[0], sg[1], sg[2], sg[3]);
    hd[i] = make_float4(sg[4], sg[5], 0.f, 0.f);
    host_store_pos(c, pos + 3 * i, ha[i], hd[i]);
  }
  int64_t k = 0;
  for (int b = 0; b < n_bodies; ++b) {
    for (int64_t q = 0; q < bodies[b].n_markers; ++q, ++k) {
      const float* l = bodies[b].marker_local + 3 * q;
      uint32_t bb = (uint32_t)b;
      float bf;
      std::memcpy(&bf, &bb, 4);
      hl[k] = make_float4(l[0], l[1], l[2], bf);
      uint32_t aux = crm::kMarker | ((uint32_t)b << 2);
      float auxf;
      std::memcpy(&auxf, &aux, 4);
      ha[n_soil + k] = make_float4(l[0], l[1], l[2], (float)P.rho0);
      hb[n_soil + k] = make_float4(0.f, 0.f, 0.f, auxf);
      hc[n_soil + k] = make_float4(0.f, 0.f, 0.f, 0.f);
      hd[n_soil + k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  c->h_bodies.resize((size_t)(n_bodies > 0 ? n_bodies : 1));
  for (int b = 0; b < n_bodies; ++b) {
    Body& B = c->h_bodies[b];
    std::memset(&B, 0, sizeof(Body));
    B.R[0] = B.R[4] = B.R[8] = 1.0;
    for (int a = 0; a < 3; ++a) B.half[a] = bodies[b].active_half[a];
    B.has_box = (B.half[0] > 0.0 || B.half[1] > 0.0 || B.half[2] > 0.0) ? 1 : 0;
    B.place = 1;
    set_box_bounds(B, g);
  }

  const int64_t nbk = crm::compact_tmp_elems(n_total);
  bool ok = alloc_n(c, c->m_a, n_total) && alloc_n(c, c->m_b, n_total) && alloc_n(c, c->m_c, n_total) &&
            alloc_n(c, c->m_d, n_total) && alloc_n(c, c->local, nm) && alloc_n(c, c->flags, crm::flags_padded(n_total)) &&
            alloc_n(c, c->proc_ids, n_total) && alloc_n(c, c->d_bodies, n_bodies > 0 ? n_bodies : 1) &&
            alloc_n(c, c->ctmp, nbk) &&
            alloc_n(c, c->cell_cnt, M) && alloc_n(c, c->cell_start, M + 1) &&
            alloc_n(c, c->cell_tmp, (int64_t)crm::scan_tmp_elems(M)) && alloc_n(c, c->d_counts, 8) &&
            alloc_n(c, c->d_mat, crm::kMaxMaterials) && alloc_n(c, c->contrib, 6 * nm) &&
            alloc_n(c, c->d_bstart, n_bodies + 1);
  if (ok && params->active_domains)
    ok = alloc_n(c, c->m_key, n_total * crm::key_words(c->grid.cell != 0));
  {
    // the block-order table bound: every rebuild window lies in the domain's grid
    const int64_t w = crm::order_width();
    const int64_t ord = (c->grid.gdim[0] + w - 1) / w * (int64_t)c->grid.gdim[1] * c->grid.gdim[2];
    if (ok && n_soil > 0 && ord <= (int64_t(1) << 26)) {
      ok = alloc_n(c, c->bperm, crm::soil_block_count(n_soil) + 1) && alloc_n(c, c->ord_cnt, ord) &&
           alloc_n(c, c->ord_first, ord) && alloc_n(c, c->ord_base, ord + 1) &&
           alloc_n(c, c->ord_scan, (int64_t)crm::scan_tmp_elems(ord));
      if (ok) c->ord_cap = ord;
    }
  }
  // the index's arrays scale with the domain's coarse cells: a domain far
  // larger than the particles it holds tests all N instead
  int32_t cd[3];
  const int64_t coarse = crm::coarse_cells(c->grid, cd);
  if (ok && params->active_domains && !params->activity_scan &&
      coarse <= std::max<int64_t>(n_total, int64_t(1) << 20)) {
    c->ix_M = crm::coarse_cells(c->grid, c->ix_cd);
    c->mcap = params->moved_cap > 0 ? params->moved_cap : std::max<int64_t>(int64_t(1) << 14, n_total / 32);
    ok = alloc_n(c, c->ix_start, c->ix_M + 1) && alloc_n(c, c->ix_fill, c->ix_M) &&
         alloc_n(c, c->ix_scan, (int64_t)crm::scan_tmp_elems(c->ix_M)) && alloc_n(c, c->ix_ids, n_total) &&
         alloc_n(c, c->ix_visit, c->ix_M) && alloc_n(c, c->moved, crm::flags_padded(n_total)) &&
         alloc_n(c, c->mlist, c->mcap) &&
         hipHostMalloc((void**)&c->h_visit_pin, sizeof(uint32_t) * (size_t)c->ix_M, hipHostMallocDefault) == hipSuccess;
    c->ix_on = ok;
    c->h_visit.reserve((size_t)std::min<int64_t>(c->ix_M, 1 << 16));
  }
  if (!ok) {
    release(c);
    return fail(nullptr, CRM_E_NOMEM, "device allocation failed");
  }
  if (hipHostMalloc((void**)&c->h_counts, sizeof(uint64_t) * 8, hipHostMallocDefault) != hipSuccess) {
    c->h_counts = nullptr;
    release(c);
    return fail(nullptr, CRM_E_NOMEM, "pinned allocation failed");
  }
  {
    const size_t nbp = (size_t)(n_bodies > 0 ? n_bodies : 1);
    if (hipHostMalloc((void**)&c->h_bpin, sizeof(Body) * nbp, hipHostMallocDefault) != hipSuccess) c->h_bpin = nullptr;
    // the force sums go straight to host memory: pinned, mapped, coherent;
    // after them one counter per body (moved by each reduction)
    if (hipHostMalloc((void**)&c->h_fpin, sizeof(double) * 7 * nbp, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&c->d_fmap, c->h_fpin, 0) != hipSuccess) {
      if (c->h_fpin) (void)hipHostFree(c->h_fpin);
      c->h_fpin = nullptr;
    } else {
      std::memset(c->h_fpin, 0, sizeof(double) * 7 * nbp);
      c->h_fseq = reinterpret_cast<volatile uint64_t*>(c->h_fpin + 6 * nbp);
      c->d_fseq = reinterpret_cast<uint64_t*>(c->d_fmap + 6 * nbp);
    }
    if (!c->h_bpin || !c->h_fpin || hipEventCreateWithFlags(&c->bpin_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fpin_ev, hipEventDisableTiming) != hipSuccess) {
      release(c);
      return fail(nullptr, CRM_E_NOMEM, "pinned allocation failed");
    }
  }
  if (params->skin > 0.0) {
    if (!alloc_n(c, c->d_disp, 1) || hipHostMalloc((void**)&c->h_disp, 4, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->disp_ev, hipEventDisableTiming) != hipSuccess) {
      c->h_disp = nullptr;
      release(c);
      return fail(nullptr, CRM_E_NOMEM, "displacement tracking allocation failed");
    }
  }
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  const size_t f4 = sizeof(float4) * (size_t)n_total;
  if (e == hipSuccess) e = hipMemcpyAsync(c->m_a, ha.data(), f4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->m_b, hb.data(), f4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->m_c, hc.data(), f4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->m_d, hd.data(), f4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = crm::key_fill(c->m_a, c->m_d, n_total, c->grid.cell != 0, c->m_key, s);
  if (e == hipSuccess && nm > 0)
    e = hipMemcpyAsync(c->local, hl.data(), sizeof(float4) * (size_t)nm, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d_bodies, c->h_bodies.data(), sizeof(Body) * c->h_bodies.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->flags, 0, (size_t)crm::flags_padded(n_total), s);
  std::vector<int64_t> bstart((size_t)n_bodies + 1, 0);
  for (int b = 0; b < n_bodies; ++b) bstart[b + 1] = bstart[b] + bodies[b].n_markers;
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d_bstart, bstart.data(), sizeof(int64_t) * bstart.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nm > 0) e = hipMemsetAsync(c->contrib, 0, sizeof(double) * 6 * (size_t)nm, s);
  c->h_nmark.resize((size_t)n_bodies);
  for (int b = 0; b < n_bodies; ++b) c->h_nmark[b] = bodies[b].n_markers;
  c->h_bstart = bstart;
  c->h_bodies_next = c->h_bodies;
  c->plan_cap = nm / crm::reduce_chunk() + n_bodies + 2;
  c->plan_lo.resize((size_t)c->plan_cap);
  c->plan_hi.resize((size_t)c->plan_cap);
  c->plan_first.resize((size_t)n_bodies + 1);
  c->plan_r.resize((size_t)n_bodies + 1);
  c->h_mattab.assign(1, make_float4((float)P.mu_s, (float)P.mu_2, (float)P.cohesion, (float)(-P.cohesion / P.mu_s)));
  {
    int64_t *dlo = nullptr, *dhi = nullptr;
    int32_t* dfirst = nullptr;
    double* dpart = nullptr;
    if (!(alloc_n(c, dlo, c->plan_cap) && alloc_n(c, dhi, c->plan_cap) && alloc_n(c, dfirst, n_bodies + 1) &&
          alloc_n(c, dpart, 6 * c->plan_cap) && alloc_n(c, c->d_branges, n_bodies + 1))) {
      release(c);
      return fail(nullptr, CRM_E_NOMEM, "device allocation failed");
    }
    c->body_plan.lo = dlo;
    c->body_plan.hi = dhi;
    c->body_plan.first = dfirst;
    c->body_plan.partial = dpart;
  }
  if (e == hipSuccess && n_bodies > 0 && fill_plan(c, bstart.data(), n_bodies, c->body_plan, c->plan_cap) != CRM_OK) {
    std::string m2 = c->err;
    release(c);
    return fail(nullptr, CRM_E_DEVICE, m2);
  }
  c->plan_all = true;
  c->kbase = n_soil;
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_mat, c->h_mattab.data(), sizeof(float4), hipMemcpyHostToDevice, s);
  c->phys.mat = c->d_mat;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    std::string m2 = std::string("upload failed: ") + hipGetErrorString(e);
    release(c);
    return fail(nullptr, CRM_E_DEVICE, m2);
  }
  *out = c;
  return CRM_OK;
}

crm_status crm_set_bodies(crm_ctx* c, int32_t nb, const double* pos, const double* quat, const double* linvel,
                          const double* angvel, const double* linacc, const double* angacc) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (nb != c->nb) return fail(c, CRM_E_INVALID, "nb differs from crm_init");
  if (nb == 0) return CRM_OK;
  if (!pos || !quat) return fail(c, CRM_E_INVALID, "pos and quat are required");
  std::vector<Body>& hb = c->h_bodies_next;   // sized at crm_init: no allocation here
  std::copy(c->h_bodies.begin(), c->h_bodies.end(), hb.begin());
  for (int b = 0; b < nb; ++b) {
    Body& B = hb[b];
    const double* arrs[] = {pos + 3 * b, linvel ? linvel + 3 * b : nullptr, angvel ? angvel + 3 * b : nullptr,
                            linacc ? linacc + 3 * b : nullptr, angacc ? angacc + 3 * b : nullptr};
    for (const double* a : arrs)
      if (a && !finite3(a)) return fail(c, CRM_E_INVALID, "non-finite body state");
    const double* q = quat + 4 * b;
    if (!(std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]) && std::isfinite(q[3])))
      return fail(c, CRM_E_INVALID, "non-finite quaternion");
    for (int a = 0; a < 3; ++a) {
      B.X[a] = pos[3 * b + a];
      B.V[a] = linvel ? linvel[3 * b + a] : 0.0;
      B.W[a] = angvel ? angvel[3 * b + a] : 0.0;
      B.A[a] = linacc ? linacc[3 * b + a] : 0.0;
      B.Al[a] = angacc ? angacc[3 * b + a] : 0.0;
    }
    quat_to_R(q, B.R);
    B.has_acc = (linacc || angacc) ? 1 : 0;
    set_box_bounds(B, c->grid);
    const Body& W = c->wplaced[b];
    B.place = (!c->wplaced_ok || std::memcmp(B.X, W.X, sizeof(B.X)) != 0 || std::memcmp(B.R, W.R, sizeof(B.R)) != 0 ||
               std::memcmp(B.V, W.V, sizeof(B.V)) != 0 || std::memcmp(B.W, W.W, sizeof(B.W)) != 0) ? 1 : 0;
  }
  hipError_t e = hipSuccess;
  if (nb <= crm::kBodyPack) {
    // a few bodies travel in a kernel's arguments
    e = crm::put_bodies(hb.data(), nb, c->d_bodies, c->stream);
  } else {
    // the staging buffer is reused once its last upload has been read
    e = c->bpin_pending ? hipEventSynchronize(c->bpin_ev) : hipSuccess;
    if (e == hipSuccess) {
      std::memcpy(c->h_bpin, hb.data(), sizeof(Body) * (size_t)nb);
      e = hipMemcpyAsync(c->d_bodies, c->h_bpin, sizeof(Body) * (size_t)nb, hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(c->bpin_ev, c->stream);
    if (e == hipSuccess) c->bpin_pending = true;
  }
  if (e != hipSuccess) return fail(c, CRM_E_DEVICE, std::string("body upload: ") + hipGetErrorString(e));
  c->h_bodies.swap(hb);
  return CRM_OK;
}

crm_status crm_set_materials(crm_ctx* c, int32_t n_mat, const double* mu_s, const double* mu_2,
                             const double* cohesion, const uint16_t* material) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (c->stepped || c->rebuilds > 0) return fail(c, CRM_E_STATE, "materials must be set before the first step");
  if (n_mat < 1 || n_mat > crm::kMaxMaterials) return fail(c, CRM_E_INVALID, "n_mat out of range");
  if (!mu_s || !mu_2 || !cohesion || (c->n_soil > 0 && !material)) return fail(c, CRM_E_INVALID, "NULL argument");
  std::vector<float4> tab((size_t)n_mat);
  for (int m = 0; m < n_mat; ++m) {
    if (!(std::isfinite(mu_s[m]) && mu_s[m] > 0.0)) return fail(c, CRM_E_INVALID, "mu_s must be > 0");
    if (!(std::isfinite(mu_2[m]) && mu_2[m] >= 0.0)) return fail(c, CRM_E_INVALID, "mu_2 must be >= 0");
    if (!(std::isfinite(cohesion[m]) && cohesion[m] >= 0.0)) return fail(c, CRM_E_INVALID, "cohesion must be >= 0");
    tab[m] = make_float4((float)mu_s[m], (float)mu_2[m], (float)cohesion[m], (float)(-cohesion[m] / mu_s[m]));
  }
  for (int64_t i = 0; i < c->n_soil; ++i)
    if (material[i] >= n_mat) return fail(c, CRM_E_INVALID, "material id out of range");
  hipStream_t s = c->stream;
  const size_t n = (size_t)c->n_soil;
  std::vector<float4> hb(n);
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(hb.data(), c->m_b, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  for (size_t i = 0; i < n; ++i) {
    uint32_t aux;
    std::memcpy(&aux, &hb[i].w, 4);
    aux = (aux & 3u) | ((uint32_t)material[i] << 2);
    std::memcpy(&hb[i].w, &aux, 4);
  }
  if (n > 0) HIPCHK(c, hipMemcpyAsync(c->m_b, hb.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_mat, tab.data(), sizeof(float4) * (size_t)n_mat, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->n_mat = n_mat;
  c->h_mattab = tab;
  c->h_mat.assign(material, material + c->n_soil);
  return CRM_OK;
}

crm_status crm_step(crm_ctx* c, int32_t n_steps) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (n_steps < 0) return fail(c, CRM_E_INVALID, "n_steps must be >= 0");
  if (n_steps > 0) c->rec_valid = false;
  for (int32_t k = 0; k < n_steps; ++k) {
    st = one_step(c);
    if (st != CRM_OK) return st;
  }
  return CRM_OK;
}

crm_status crm_step_noalloc(crm_ctx* c, int32_t n_steps) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (n_steps < 0) return fail(c, CRM_E_INVALID, "n_steps must be >= 0");
  if (!c->scratch) return fail(c, CRM_E_STATE, "no scratch address for this context's device");
  if (!c->A.a) return fail(c, CRM_E_NOMEM, "the working set is not allocated yet (a call that may allocate is needed)");
  const ScratchLayout L = scratch_layout(c);
  if (L.bytes > crm::kScratchBytes)
    return fail(c, CRM_E_INVALID, "the context needs " + std::to_string(L.bytes) + " bytes of scratch, more than the " +
                                      std::to_string(crm::kScratchBytes) + " the library holds per device");
  if (n_steps > 0) c->rec_valid = false;
  const bool prof = c->prof;
  c->prof = false;   // timing events are created on demand: not recorded here
  {
    NoAllocScope scope(c, L);
    for (int32_t k = 0; k < n_steps; ++k) {
      // direct launches: capturing or instantiating a graph allocates
      if (rebuild_due(c)) {
        st = rebuild(c);
        if (st != CRM_OK) break;
      }
      st = launch_step(c, c->stream, false);
      if (st != CRM_OK) break;
      note_placement(c);
      st = track_displacement(c);
      if (st != CRM_OK) break;
      c->step += 1;
      c->stepped = true;
    }
  }
  c->prof = prof;
  return st;
}

crm_status crm_record(crm_ctx* c, int32_t n_steps) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (n_steps < 1) return fail(c, CRM_E_INVALID, "n_steps must be >= 1");
  if (c->prm.active_domains) return fail(c, CRM_E_UNSUPPORTED, "the reverse sweep covers runs without active domains");
  if (c->prm.skin > 0.0) c->force_rebuild = true;   // Verlet lists: the record starts with a rebuild
  if (!rebuild_due(c)) return fail(c, CRM_E_STATE, "a record starts at a list rebuild (step mod ps_freq = 0)");
  const int64_t ps = c->prm.ps_freq;
  const int64_t segs = (int64_t)n_steps / ps + 2;
  c->rec_valid = false;
  dfree(c, c->rec_snap);
  c->rec_snap = nullptr;
  c->rec_snap_cap = 0;
  dfree(c, c->rec_forces);
  c->rec_forces = nullptr;
  if (!alloc_n(c, c->rec_snap, segs * 4 * c->n_total)) return fail(c, CRM_E_NOMEM, "record snapshot allocation failed");
  c->rec_snap_cap = segs;
  const int64_t nf = 6 * (int64_t)c->nb;
  if (nf > 0 && !alloc_n(c, c->rec_forces, (int64_t)n_steps * nf))
    return fail(c, CRM_E_NOMEM, "record force allocation failed");
  c->rec_bodies = c->h_bodies;
  c->rec_step0 = c->step;
  c->rec_seg.clear();
  c->recording = true;
  for (int32_t k = 0; k < n_steps; ++k) {
    st = one_step(c);
    if (st == CRM_OK && nf > 0) {
      const hipError_t e = crm::copy_f64(c->rec_forces + (size_t)k * (size_t)nf, c->d_fmap, nf, c->stream);
      if (e != hipSuccess) st = fail(c, CRM_E_DEVICE, std::string("record forces: ") + hipGetErrorString(e));
    }
    if (st != CRM_OK) {
      c->recording = false;
      return st;
    }
  }
  c->recording = false;
  c->rec_n = n_steps;
  c->rec_valid = true;
  return CRM_OK;
}

crm_status crm_record_forces(crm_ctx* c, double* force, double* torque) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (!c->rec_valid) return fail(c, CRM_E_STATE, "no recorded run (crm_record)");
  const int64_t nb = c->nb, n = (int64_t)c->rec_n;
  if (nb == 0) return CRM_OK;
  if (!force || !torque) return fail(c, CRM_E_INVALID, "force and torque are required");
  std::vector<double> h((size_t)(6 * nb * n));
  HIPCHK(c, hipMemcpyAsync(h.data(), c->rec_forces, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t k = 0; k < n * nb; ++k)
    for (int a = 0; a < 3; ++a) {
      force[3 * k + a] = h[(size_t)(6 * k + a)];
      torque[3 * k + a] = h[(size_t)(6 * k + 3 + a)];
    }
  for (double v : h)
    if (!std::isfinite(v)) return fail(c, CRM_E_NONFINITE, "non-finite body force or torque in the record");
  return CRM_OK;
}

crm_status crm_adjoint(crm_ctx* c, const double* lam_pos, const float* lam_vel, const float* lam_sigma,
                       const float* lam_rho, const double* lam_force, const double* lam_torque, double* out_pos,
                       float* out_vel, float* out_sigma, float* out_rho, double* out_params) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (!c->rec_valid) return fail(c, CRM_E_STATE, "no recorded run (crm_record) to reverse");
  if (c->step != c->rec_step0 + c->rec_n) return fail(c, CRM_E_STATE, "the context has moved since crm_record");
  hipStream_t s = c->stream;
  const int64_t ns = c->n_soil, nt = c->n_total;
  const int32_t nb = c->nb;
  const int64_t nseg = (int64_t)c->rec_seg.size();
  int64_t seg_max = 0;
  for (int64_t g = 0; g < nseg; ++g) {
    const int64_t k1 = g + 1 < nseg ? c->rec_seg[g + 1] : c->rec_n;
    seg_max = std::max<int64_t>(seg_max, k1 - c->rec_seg[g]);
  }
  const bool force_seed = (lam_force || lam_torque) && nb > 0;
  const int32_t ngrp = c->n_mat + 1;   // materials, then the markers
  std::vector<void*> tmp;
  auto take = [&](auto*& p, int64_t n) {
    bool ok = alloc_n(c, p, n);
    if (ok) tmp.push_back((void*)p);
    return ok;
  };
  auto done = [&](crm_status r) {
    (void)hipStreamSynchronize(s);
    for (void* p : tmp) dfree(c, p);
    return r;
  };
  auto planes = [&](Planes& P, int64_t n) {
    return take(P.a, n) && take(P.b, n) && take(P.c, n) && take(P.d, n);
  };
  Planes Ln{}, Lm{}, E{}, Lid{};
  float* pg = nullptr;
  double *pid = nullptr, *fseed = nullptr, *ptmp = nullptr, *gsum = nullptr;
  int32_t* perm = nullptr;
  std::vector<StepRecord> recs((size_t)seg_max);
  bool ok = planes(Ln, nt) && planes(Lm, nt) && planes(E, nt) && planes(Lid, ns > 0 ? ns : 1) && take(pg, 5 * nt) &&
            take(pid, 6 * nt) && take(ptmp, 6 * nt) && take(gsum, 6 * ngrp) && take(perm, nt) &&
(!force_seed || take(fseed, (int64_t)c->rec_n * nb * 6));
  for (auto& r : recs)
    ok = ok && planes(r.yn, nt) && planes(r.ym, nt) && take(r.t1.l0, nt) && take(r.t1.l1, nt) &&
         take(r.t1.l2, nt) && take(r.t2.l0, nt) && take(r.t2.l1, nt) && take(r.t2.l2, nt) && take(r.t2.t0, nt) &&
         take(r.t2.t1, nt);
  if (!ok) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
  // seeds on the recorded end state (particle-id order): the caller's arrays
  // as they are, packed on the device; and on the body forces
  {
    double* dpos = nullptr;
    float *dvel = nullptr, *dsig = nullptr, *drho = nullptr;
    if (ns > 0) {
      if (lam_pos && !take(dpos, 3 * ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (lam_vel && !take(dvel, 3 * ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (lam_sigma && !take(dsig, 6 * ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (lam_rho && !take(drho, ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (dpos) HIPCHK(c, hipMemcpyAsync(dpos, lam_pos, sizeof(double) * 3 * ns, hipMemcpyHostToDevice, s));
      if (dvel) HIPCHK(c, hipMemcpyAsync(dvel, lam_vel, sizeof(float) * 3 * ns, hipMemcpyHostToDevice, s));
      if (dsig) HIPCHK(c, hipMemcpyAsync(dsig, lam_sigma, sizeof(float) * 6 * ns, hipMemcpyHostToDevice, s));
      if (drho) HIPCHK(c, hipMemcpyAsync(drho, lam_rho, sizeof(float) * ns, hipMemcpyHostToDevice, s));
      HIPCHK(c, crm::adj_pack(ns, dpos, dvel, dsig, drho, Lid, s));
    }
    if (force_seed) {
      std::vector<double> f((size_t)c->rec_n * nb * 6, 0.0);
      for (int64_t k = 0; k < (int64_t)c->rec_n * nb; ++k)
        for (int a = 0; a < 3; ++a) {
          f[6 * k + a] = lam_force ? lam_force[3 * k + a] : 0.0;
          f[6 * k + 3 + a] = lam_torque ? lam_torque[3 * k + a] : 0.0;
        }
      HIPCHK(c, hipMemcpyAsync(fseed, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice, s));
    }
    HIPCHK(c, hipMemsetAsync(pg, 0, sizeof(float) * 5 * (size_t)nt, s));
    HIPCHK(c, hipMemsetAsync(pid, 0, sizeof(double) * 6 * (size_t)nt, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  const std::vector<Body> cur_bodies = c->h_bodies;
  auto set_bodies_dev = [&](const std::vector<Body>& B) -> crm_status {
    HIPCHK(c, hipMemcpyAsync(c->d_bodies, B.data(), sizeof(Body) * B.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    c->h_bodies = B;
    return CRM_OK;
  };
  auto restore = [&](int64_t g) -> crm_status {
    const size_t n = (size_t)nt;
    const float4* src = c->rec_snap + (size_t)g * 4 * n;
    float4* dst[4] = {c->m_a, c->m_b, c->m_c, c->m_d};
    for (int q = 0; q < 4; ++q)
      HIPCHK(c, hipMemcpyAsync(dst[q], src + q * n, sizeof(float4) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, crm::key_fill(c->m_a, c->m_d, (int64_t)n, c->grid.cell != 0, c->m_key, s));
    c->ix_valid = false;
    c->working_valid = false;
    c->force_rebuild = true;
    c->place_all = true;
    c->step = c->rec_step0 + c->rec_seg[g];
    c->fpin_step = -1;
    return CRM_OK;
  };
  // the gathers below walk every soil row's slots: the replays' rebuilds write
  // them all (until this call returns, on every path)
  struct FullLists {
    crm_ctx* c;
    ~FullLists() { c->full_lists = false; }
  } full_lists_scope{c};
  c->full_lists = true;
  st = set_bodies_dev(c->rec_bodies);
  if (st != CRM_OK) return done(st);
  const Phys& P = c->phys;
  for (int64_t g = nseg - 1; g >= 0; --g) {
    const int64_t k0 = c->rec_seg[g], k1 = g + 1 < nseg ? c->rec_seg[g + 1] : c->rec_n;
    st = restore(g);
    if (st != CRM_OK) return done(st);
    for (int64_t k = k0; k < k1; ++k) {
      st = one_step(c, &recs[k - k0]);
      if (st != CRM_OK) return done(st);
    }
    HIPCHK(c, crm::adj_to_slots(c->frows, c->n_frows, c->slot_id, Lid, Ln, s));
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const StepRecord& R = recs[k - k0];
      const double* fs = force_seed ? fseed + (size_t)k * nb * 6 : nullptr;
      // stage 2 (y* = y_n + dt f(y_mid), return mapping, body forces of y_mid)
      HIPCHK(c, crm::adj_local2(c->frows, c->n_frows, Ln, Lm, E, R.yn, R.ym, R.t2, P, pg, s));
      HIPCHK(c, crm::adj_marker(R.ym, E, c->mrows, c->n_mrows, c->off_m, c->nbr_m, c->d_bodies, fs, P, pg, s));
      HIPCHK(c, crm::adj_gather(R.ym, E, c->frows, c->n_frows, c->off_f, c->nbr_f, P, Lm, pg, s));
      // stage 1 (y_mid = y_n + dt/2 f(y_n))
      HIPCHK(c, crm::adj_local1(c->frows, c->n_frows, Ln, Lm, E, R.yn, R.t1, P, pg, s));
      HIPCHK(c, crm::adj_marker(R.yn, E, c->mrows, c->n_mrows, c->off_m, c->nbr_m, c->d_bodies, nullptr, P, pg, s));
      HIPCHK(c, crm::adj_gather(R.yn, E, c->frows, c->n_frows, c->off_f, c->nbr_f, P, Ln, pg, s));
    }
    HIPCHK(c, crm::adj_to_ids(c->frows, c->n_frows, c->slot_id, Ln, Lid, s));
    HIPCHK(c, crm::adj_params_to_ids(c->n_proc, c->slot_id, pg, pid, s));
  }
  // parameter sums per material (and the markers) in a fixed order
  std::vector<int32_t> hperm((size_t)nt);
  std::vector<int64_t> hstart((size_t)ngrp + 1, 0);
  {
    std::vector<int64_t> cnt((size_t)ngrp, 0);
    for (int64_t i = 0; i < ns; ++i) cnt[c->h_mat.empty() ? 0 : c->h_mat[i]] += 1;
    cnt[ngrp - 1] = nt - ns;
    for (int32_t g = 0; g < ngrp; ++g) hstart[g + 1] = hstart[g] + cnt[g];
    std::vector<int64_t> pos(hstart.begin(), hstart.end() - 1);
    for (int64_t i = 0; i < ns; ++i) hperm[pos[c->h_mat.empty() ? 0 : c->h_mat[i]]++] = (int32_t)i;
    for (int64_t i = ns; i < nt; ++i) hperm[pos[ngrp - 1]++] = (int32_t)i;
  }
  HIPCHK(c, hipMemcpyAsync(perm, hperm.data(), sizeof(int32_t) * hperm.size(), hipMemcpyHostToDevice, s));
  crm::SegPlan gplan;
  st = make_plan(c, hstart, gplan, &tmp);
  if (st != CRM_OK) return done(st);
  HIPCHK(c, crm::adj_params_permute(nt, perm, pid, ptmp, s));
  HIPCHK(c, crm::segment_reduce(ptmp, gplan, gsum, s));
  std::vector<double> hsum((size_t)6 * ngrp);
  HIPCHK(c, hipMemcpyAsync(hsum.data(), gsum, sizeof(double) * hsum.size(), hipMemcpyDeviceToHost, s));
  // adjoint of the recorded start state: unpacked on the device, copied into
  // the caller's arrays
  {
    double* dpos = nullptr;
    float *dvel = nullptr, *dsig = nullptr, *drho = nullptr;
    uint32_t* dbad = nullptr;
    if (!take(dbad, 1)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
    HIPCHK(c, crm::fill_u32(dbad, 0u, 1, s));
    if (ns > 0) {
      if (out_pos && !take(dpos, 3 * ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (out_vel && !take(dvel, 3 * ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (out_sigma && !take(dsig, 6 * ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      if (out_rho && !take(drho, ns)) return done(fail(c, CRM_E_NOMEM, "adjoint allocation failed"));
      HIPCHK(c, crm::adj_unpack(ns, Lid, dpos, dvel, dsig, drho, dbad, s));
      if (dpos) HIPCHK(c, hipMemcpyAsync(out_pos, dpos, sizeof(double) * 3 * ns, hipMemcpyDeviceToHost, s));
      if (dvel) HIPCHK(c, hipMemcpyAsync(out_vel, dvel, sizeof(float) * 3 * ns, hipMemcpyDeviceToHost, s));
      if (dsig) HIPCHK(c, hipMemcpyAsync(out_sigma, dsig, sizeof(float) * 6 * ns, hipMemcpyDeviceToHost, s));
      if (drho) HIPCHK(c, hipMemcpyAsync(out_rho, drho, sizeof(float) * ns, hipMemcpyDeviceToHost, s));
    }
    uint32_t hbad = 0;
    HIPCHK(c, hipMemcpyAsync(&hbad, dbad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    bool finite = hbad == 0;
    if (out_params) {
      double dG = 0.0, dK = 0.0;
      for (int32_t g = 0; g < ngrp; ++g) {
        dG += hsum[6 * g];
        dK += hsum[6 * g + 1];
      }
      const double E_ = c->prm.E, nu = c->prm.nu;
      out_params[0] = dG / (2.0 * (1.0 + nu)) + dK / (3.0 * (1.0 - 2.0 * nu));
      out_params[1] = -dG * E_ / (2.0 * (1.0 + nu) * (1.0 + nu)) + dK * 2.0 * E_ / (3.0 * (1.0 - 2.0 * nu) * (1.0 - 2.0 * nu));
      for (int32_t m = 0; m < c->n_mat; ++m)
        for (int a = 0; a < 3; ++a) out_params[2 + 3 * m + a] = hsum[6 * m + 2 + a];
      for (int k = 0; k < 2 + 3 * c->n_mat; ++k) finite = finite && std::isfinite(out_params[k]);
    }
    if (!finite) st = fail(c, CRM_E_NONFINITE, "non-finite adjoint");
  }
  // back to the recorded end state: the last segment again, forward
  if (st == CRM_OK) {
    const int64_t g = nseg - 1;
    st = restore(g);
    for (int64_t k = c->rec_seg[g]; st == CRM_OK && k < c->rec_n; ++k) st = one_step(c);
  }
  if (st == CRM_OK) st = set_bodies_dev(cur_bodies);
  return done(st);
}

crm_status crm_get_forces(crm_ctx* c, int32_t nb, double* force, double* torque) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (nb != c->nb) return fail(c, CRM_E_INVALID, "nb differs from crm_init");
  if ((!force || !torque) && nb > 0) return fail(c, CRM_E_INVALID, "force and torque are required");
  if (!c->stepped) return fail(c, CRM_E_STATE, "no step taken yet");
  if (nb == 0) return CRM_OK;
  // the last step's reduction wrote the sums into h_fpin (mapped host memory)
  if (c->fpin_step == c->step) {
    // its counters, polled; the stream's state is looked at now and then, so
    // that a device error ends the wait
    for (uint32_t it = 1;; ++it) {
      bool done = true;
      for (int b = 0; b < nb && done; ++b) done = c->h_fseq[b] == c->fseq;
      if (done) break;
      if ((it & 1023u) == 0) {
        const hipError_t e = hipStreamQuery(c->stream);
        if (e == hipSuccess) {
          for (int b = 0; b < nb; ++b)
            if (c->h_fseq[b] != c->fseq) return fail(c, CRM_E_DEVICE, "body sums not written by the finished stream");
          break;
        }
        if (e != hipErrorNotReady) return fail(c, CRM_E_DEVICE, std::string("force read: ") + hipGetErrorString(e));
      }
    }
  } else {
    HIPCHK(c, hipEventRecord(c->fpin_ev, c->stream));
    HIPCHK(c, poll_event(c->fpin_ev));
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  const double* h = c->h_fpin;
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      force[3 * b + a] = h[6 * b + a];
      torque[3 * b + a] = h[6 * b + 3 + a];
    }
  for (int k = 0; k < 6 * nb; ++k)
    if (!std::isfinite(h[k])) return fail(c, CRM_E_NONFINITE, "non-finite body force or torque");
  return CRM_OK;
}

crm_status crm_cosim_step(crm_ctx* c, int32_t nb, const double* pos, const double* quat, const double* linvel,
                          const double* angvel, const double* linacc, const double* angacc, double* force,
                          double* torque) {
  crm_status st = crm_set_bodies(c, nb, pos, quat, linvel, angvel, linacc, angacc);
  if (st != CRM_OK) return st;
  st = crm_step(c, 1);
  if (st != CRM_OK) return st;
  return crm_get_forces(c, nb, force, torque);
}

crm_status crm_get_state(crm_ctx* c, double* pos, float* vel, float* sigma, float* rho) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  hipStream_t s = c->stream;
  if (c->working_valid) {
    crm_status st0 = scatter_back(c);
    if (st0 != CRM_OK) return st0;
  }
  {
    crm_status st0 = place_master_markers(c);
    if (st0 != CRM_OK) return st0;
  }
  const size_t n = (size_t)c->n_total;
  std::vector<float4> ha(n), hb(n), hc(n), hd(n);
  HIPCHK(c, hipMemcpyAsync(ha.data(), c->m_a, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hb.data(), c->m_b, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hc.data(), c->m_c, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hd.data(), c->m_d, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i) {
    if (pos) host_abs_pos(c, ha[i], hd[i], pos + 3 * i);
    if (rho) rho[i] = ha[i].w;
    if (vel) { vel[3 * i] = hb[i].x; vel[3 * i + 1] = hb[i].y; vel[3 * i + 2] = hb[i].z; }
    if (sigma) {
      sigma[6 * i] = hc[i].x; sigma[6 * i + 1] = hc[i].y; sigma[6 * i + 2] = hc[i].z;
      sigma[6 * i + 3] = hc[i].w; sigma[6 * i + 4] = hd[i].x; sigma[6 * i + 5] = hd[i].y;
    }
  }
  return CRM_OK;
}

crm_status crm_set_state(crm_ctx* c, const double* pos, const float* vel, const float* sigma, const float* rho) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  const int64_t n = c->n_soil;
  if (pos)
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(pos[i])) return fail(c, CRM_E_INVALID, "non-finite position");
  hipStream_t s = c->stream;
  if (c->working_valid) {
    crm_status st0 = scatter_back(c);
    if (st0 != CRM_OK) return st0;
  }
  std::vector<float4> ha((size_t)n), hb((size_t)n), hc((size_t)n), hd((size_t)n);
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(ha.data(), c->m_a, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(hb.data(), c->m_b, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(hc.data(), c->m_c, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(hd.data(), c->m_d, sizeof(float4) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  for (int64_t i = 0; i < n; ++i) {
    if (pos) host_store_pos(c, pos + 3 * i, ha[i], hd[i]);
    if (rho) ha[i].w = rho[i];
    if (vel) { hb[i].x = vel[3 * i]; hb[i].y = vel[3 * i + 1]; hb[i].z = vel[3 * i + 2]; }
    if (sigma) {
      hc[i] = make_float4(sigma[6 * i], sigma[6 * i + 1], sigma[6 * i + 2], sigma[6 * i + 3]);
      hd[i].x = sigma[6 * i + 4];
      hd[i].y = sigma[6 * i + 5];
    }
  }
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(c->m_a, ha.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->m_b, hb.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->m_c, hc.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->m_d, hd.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, crm::key_fill(c->m_a, c->m_d, n, c->grid.cell != 0, c->m_key, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  c->working_valid = false;
  c->force_rebuild = true;
  c->rec_valid = false;
  c->ix_valid = false;
  return CRM_OK;
}

namespace {

// Layout of a checkpoint: this header, the four master planes (n_total float4
// each), the body table (nb Body), the material table (n_mat float4) and, when
// materials were set, the material of each soil particle (n_soil uint16).
struct CkptHeader {
  char magic[8];
  uint32_t abi_version, pos_mode;
  int64_t n_total, n_soil;
  int32_t nb, n_mat;
  int64_t step;
  int32_t tile_cfg, has_mat;
  int64_t payload;   // bytes after the header
};
constexpr char kCkptMagic[8] = {'C', 'R', 'M', 'C', 'K', 'P', 'T', '1'};

size_t ckpt_payload(const crm_ctx* c, int32_t n_mat, bool has_mat) {
  return 4 * sizeof(float4) * (size_t)c->n_total + sizeof(Body) * (size_t)c->nb + sizeof(float4) * (size_t)n_mat +
         (has_mat ? sizeof(uint16_t) * (size_t)c->n_soil : 0);
}

}  // namespace

crm_status crm_checkpoint_bytes(crm_ctx* c, size_t* bytes) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (!bytes) return fail(c, CRM_E_INVALID, "bytes is NULL");
  *bytes = sizeof(CkptHeader) + ckpt_payload(c, c->n_mat, !c->h_mat.empty());
  return CRM_OK;
}

crm_status crm_save_checkpoint(crm_ctx* c, void* buf, size_t bytes) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  const bool has_mat = !c->h_mat.empty();
  const size_t need = sizeof(CkptHeader) + ckpt_payload(c, c->n_mat, has_mat);
  if (!buf || bytes < need) return fail(c, CRM_E_INVALID, "checkpoint buffer is NULL or too small");
  if (!rebuild_due(c))
    return fail(c, CRM_E_STATE, "a checkpoint is taken where the next step rebuilds the lists (step mod ps_freq = 0)");
  hipStream_t s = c->stream;
  if (c->working_valid) {
    crm_status st0 = scatter_back(c);
    if (st0 != CRM_OK) return st0;
  }
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, sizeof(h.magic));
  h.abi_version = CRM_ABI_VERSION;
  h.pos_mode = (uint32_t)c->grid.cell;
  h.n_total = c->n_total;
  h.n_soil = c->n_soil;
  h.nb = c->nb;
  h.n_mat = c->n_mat;
  h.step = c->step;
  h.tile_cfg = c->tile_cfg;
  h.has_mat = has_mat ? 1 : 0;
  h.payload = (int64_t)(need - sizeof(CkptHeader));
  char* o = static_cast<char*>(buf);
  std::memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  const size_t pl = sizeof(float4) * (size_t)c->n_total;
  const float4* planes[4] = {c->m_a, c->m_b, c->m_c, c->m_d};
  for (int q = 0; q < 4; ++q, o += pl) HIPCHK(c, hipMemcpyAsync(o, planes[q], pl, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (c->nb > 0) std::memcpy(o, c->h_bodies.data(), sizeof(Body) * (size_t)c->nb);
  o += sizeof(Body) * (size_t)c->nb;
  std::memcpy(o, c->h_mattab.data(), sizeof(float4) * (size_t)c->n_mat);
  o += sizeof(float4) * (size_t)c->n_mat;
  if (has_mat) std::memcpy(o, c->h_mat.data(), sizeof(uint16_t) * (size_t)c->n_soil);
  return CRM_OK;
}

crm_status crm_load_checkpoint(crm_ctx* c, const void* buf, size_t bytes) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  CkptHeader h{};
  if (!buf || bytes < sizeof(h)) return fail(c, CRM_E_INVALID, "not a checkpoint (too short)");
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, sizeof(h.magic)) != 0 || h.abi_version != CRM_ABI_VERSION)
    return fail(c, CRM_E_INVALID, "not a checkpoint of this library version");
  if (h.n_total != c->n_total || h.n_soil != c->n_soil || h.nb != c->nb || h.pos_mode != (uint32_t)c->grid.cell)
    return fail(c, CRM_E_INVALID, "checkpoint of another configuration (particles, bodies or position form)");
  if (h.n_mat < 1 || h.n_mat > crm::kMaxMaterials || h.step < 0 || h.tile_cfg < CRM_TILE_NONE ||
      h.tile_cfg > CRM_TILE_LARGE)
    return fail(c, CRM_E_INVALID, "corrupt checkpoint header");
  const size_t need = sizeof(h) + ckpt_payload(c, h.n_mat, h.has_mat != 0);
  if (h.payload != (int64_t)(need - sizeof(h)) || bytes < need)
    return fail(c, CRM_E_INVALID, "checkpoint size does not match its header");
  const char* o = static_cast<const char*>(buf) + sizeof(h);
  const size_t pl = sizeof(float4) * (size_t)c->n_total;
  const char* bodies = o + 4 * pl;
  const char* mattab = bodies + sizeof(Body) * (size_t)c->nb;
  const char* mats = mattab + sizeof(float4) * (size_t)h.n_mat;
  hipStream_t s = c->stream;
  HIPCHK(c, hipStreamSynchronize(s));
  float4* planes[4] = {c->m_a, c->m_b, c->m_c, c->m_d};
  for (int q = 0; q < 4; ++q) HIPCHK(c, hipMemcpyAsync(planes[q], o + q * pl, pl, hipMemcpyHostToDevice, s));
  HIPCHK(c, crm::key_fill(c->m_a, c->m_d, c->n_total, c->grid.cell != 0, c->m_key, s));
  c->ix_valid = false;
  std::vector<Body> hb((size_t)(c->nb > 0 ? c->nb : 1));
  if (c->nb > 0) std::memcpy(hb.data(), bodies, sizeof(Body) * (size_t)c->nb);
  std::vector<float4> tab((size_t)h.n_mat);
  std::memcpy(tab.data(), mattab, sizeof(float4) * (size_t)h.n_mat);
  HIPCHK(c, hipMemcpyAsync(c->d_bodies, hb.data(), sizeof(Body) * hb.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_mat, tab.data(), sizeof(float4) * tab.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->h_bodies = hb;
  c->h_mattab = tab;
  c->n_mat = h.n_mat;
  if (h.has_mat) {
    c->h_mat.resize((size_t)c->n_soil);
    std::memcpy(c->h_mat.data(), mats, sizeof(uint16_t) * (size_t)c->n_soil);
  } else {
    c->h_mat.clear();
  }
  c->step = h.step;
  c->fpin_step = -1;
  c->tile_cfg = h.tile_cfg;
  c->working_valid = false;
  c->force_rebuild = true;
  c->place_all = true;
  c->wplaced_ok = false;
  c->rec_valid = false;
  c->stepped = false;
  c->disp_pending = false;
  c->last_rebuild = h.step;
  return CRM_OK;
}

crm_status crm_get_counts(crm_ctx* c, int64_t* out) {
  if (!c || !out) return fail(c, CRM_E_INVALID, "NULL argument");
  out[0] = c->n_total;
  out[1] = c->n_soil;
  out[2] = c->n_proc;
  out[3] = c->n_frows;
  out[4] = c->n_mrows;
  out[5] = c->ent_f + c->ent_m;
  out[6] = c->cap;
  out[7] = c->step;
  out[8] = c->M;
  out[9] = c->rebuilds;
  return CRM_OK;
}

crm_status crm_debug_export(crm_ctx* c, int32_t* sorted_ids, uint32_t* cell_start, int32_t* rows, int64_t* off,
                            int32_t* nbr, int64_t cap, uint8_t* flags) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (c->rebuilds == 0 || !c->working_valid) return fail(c, CRM_E_STATE, "no valid rebuild to export");
  hipStream_t s = c->stream;
  st = complete_lists(c);
  if (st != CRM_OK) return st;
  const int64_t np = c->n_proc;
  std::vector<int32_t> sid((size_t)np);
  HIPCHK(c, hipMemcpyAsync(sid.data(), c->slot_id, sizeof(int32_t) * (size_t)np, hipMemcpyDeviceToHost, s));
  std::vector<uint32_t> wcs;
  if (cell_start) {
    if (c->Mw == c->M) {
      HIPCHK(c, hipMemcpyAsync(cell_start, c->cell_start, sizeof(uint32_t) * (size_t)(c->M + 1), hipMemcpyDeviceToHost, s));
    } else {   // a window of the domain's grid: spread its cellStart over the domain's cells below
      wcs.resize((size_t)(c->Mw + 1));
      HIPCHK(c, hipMemcpyAsync(wcs.data(), c->cell_start, sizeof(uint32_t) * wcs.size(), hipMemcpyDeviceToHost, s));
    }
  }
  if (flags) {
    if (c->ad_on)
      HIPCHK(c, hipMemcpyAsync(flags, c->flags, (size_t)c->n_total, hipMemcpyDeviceToHost, s));
    else
      std::memset(flags, 2, (size_t)c->n_total);
  }
  const bool want_lists = rows || off || nbr;
  std::vector<int32_t> fr, mr;
  std::vector<uint64_t> of, om;
  std::vector<uint32_t> ef, em;
  if (want_lists) {
    fr.resize((size_t)c->n_frows); mr.resize((size_t)c->n_mrows);
    of.resize((size_t)c->n_frows + 1); om.resize((size_t)c->n_mrows + 1);
    ef.resize((size_t)c->ent_f); em.resize((size_t)c->ent_m);
    auto cp = [&](void* d, const void* src, size_t bytes) {
      return bytes ? hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
    };
    HIPCHK(c, cp(fr.data(), c->frows, 4 * fr.size()));
    HIPCHK(c, cp(mr.data(), c->mrows, 4 * mr.size()));
    HIPCHK(c, cp(of.data(), c->off_f, 8 * of.size()));
    HIPCHK(c, cp(om.data(), c->off_m, 8 * om.size()));
    HIPCHK(c, cp(ef.data(), c->nbr_f, 4 * ef.size()));
    HIPCHK(c, cp(em.data(), c->nbr_m, 4 * em.size()));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  if (sorted_ids) std::memcpy(sorted_ids, sid.data(), sizeof(int32_t) * (size_t)np);
  if (!wcs.empty()) {
    // cellStart of a domain cell = particles in window cells before it, in the
    // common (z, y, x) order
    const Grid& w = c->wgrid;
    const int64_t X = c->grid.gdim[0], Y = c->grid.gdim[1], Z = c->grid.gdim[2];
    uint32_t running = 0;
    int64_t g = 0;
    for (int64_t z = 0; z < Z; ++z)
      for (int64_t y = 0; y < Y; ++y) {
        const bool in_zy = z >= w.org[2] && z < w.org[2] + w.dims[2] && y >= w.org[1] && y < w.org[1] + w.dims[1];
        for (int64_t x = 0; x < X; ++x, ++g) {
          if (in_zy && x >= w.org[0] && x < w.org[0] + w.dims[0]) {
            const int64_t wk = ((z - w.org[2]) * w.dims[1] + (y - w.org[1])) * w.dims[0] + (x - w.org[0]);
            cell_start[g] = wcs[(size_t)wk];
            running = wcs[(size_t)wk + 1];
          } else {
            cell_start[g] = running;
          }
        }
      }
    cell_start[c->M] = (uint32_t)np;
  }
  if (want_lists) {
    const int64_t tot = (int64_t)(of.back() + om.back());
    if (nbr && tot > cap) return fail(c, CRM_E_INVALID, "cap too small for the neighbour entries");
    int64_t row = 0, e = 0;
    auto emit = [&](const std::vector<int32_t>& rr, const std::vector<uint64_t>& oo,
                    const std::vector<uint32_t>& ee) {
      for (size_t r = 0; r < rr.size(); ++r, ++row) {
        if (rows) rows[row] = sid[(size_t)rr[r]];
        if (off) off[row] = e;
        for (uint64_t k = oo[r]; k < oo[r + 1]; ++k, ++e)
          if (nbr) nbr[e] = sid[ee[k]];
      }
    };
    emit(fr, of, ef);
    emit(mr, om, em);
    if (off) off[row] = e;
  }
  return CRM_OK;
}

crm_status crm_autotune(crm_ctx* c, int32_t config, int32_t* chosen) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (config > CRM_TILE_LARGE) return fail(c, CRM_E_INVALID, "unknown tile configuration");
  if (config >= 0) {
    // blocks the new tile cannot hold read their slots through L1
    if (crm::tile_records(config, c->grid.cell != 0) < c->nbr_skip) {
      st = complete_lists(c);
      if (st != CRM_OK) return st;
    }
    c->tile_cfg = config;
    if (chosen) *chosen = config;
    return CRM_OK;
  }
  if (!c->working_valid || c->n_frows == 0) {
    if (chosen) *chosen = c->tile_cfg;
    return c->working_valid ? CRM_OK : fail(c, CRM_E_STATE, "autotuning needs a list rebuild (take a step first)");
  }
  // stage 1 writes only y_mid, which the next step recomputes: time it on the
  // current state with each configuration (every slot in nbr_f for the blocks
  // a configuration reads through L1)
  st = complete_lists(c);
  if (st != CRM_OK) return st;
  hipStream_t s = c->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float best = 0.f;
  int32_t pick = c->tile_cfg;
  for (int32_t cfg = CRM_TILE_NONE; cfg <= CRM_TILE_LARGE; ++cfg) {
    hipError_t e = crm::fluid_stage1(c->A, c->B, c->frows, c->n_frows, c->off_f, c->nbr_f, c->phys, nullptr, c->tabs,
                                     c->tix_f, cfg, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && e == hipSuccess; ++r)
      e = crm::fluid_stage1(c->A, c->B, c->frows, c->n_frows, c->off_f, c->nbr_f, c->phys, nullptr, c->tabs,
                            c->tix_f, cfg, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(c, CRM_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
    }
    if (cfg == CRM_TILE_NONE || ms < best) {
      best = ms;
      pick = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tile_cfg = pick;
  if (chosen) *chosen = pick;
  return CRM_OK;
}

crm_status crm_set_graph(crm_ctx* c, int32_t enable) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  c->use_graph = enable != 0;
  if (!c->use_graph) drop_graph(c);
  return CRM_OK;
}

crm_status crm_set_profiling(crm_ctx* c, int32_t enable) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t mask;
  if (enable == 0 || enable == 1) mask = enable ? 0xffu : 0u;
  else if ((enable & ~0xff) == CRM_PROF_CLASSES) mask = (uint32_t)enable & 0xffu;
  else return fail(c, CRM_E_INVALID, "enable must be 0, 1 or CRM_PROF_CLASSES | class bits");
  if (mask) {
    c->prof_marks.clear();
    c->ev_used = 0;
  }
  c->prof = mask != 0;
  c->prof_mask = mask;
  return CRM_OK;
}

crm_status crm_get_profile(crm_ctx* c, double* out) {
  crm_status st = usable(c);
  if (st != CRM_OK) return st;
  if (!out) return fail(c, CRM_E_INVALID, "out is NULL");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 18; ++k) out[k] = 0.0;
  for (auto& m : c->prof_marks) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, m.second.first, m.second.second));
    const int at = m.first < 7 ? 2 * m.first : 2 * m.first + 2;   // class 7 after the pair counts
    out[at] += 1.0;
    out[at + 1] += (double)ms;
  }
  auto pairs = [&](const uint32_t* cnt, int64_t n, double& dst) -> crm_status {
    std::vector<uint32_t> h((size_t)n);
    if (n > 0) HIPCHK(c, hipMemcpy(h.data(), cnt, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost));
    double t = 0.0;
    for (uint32_t v : h) t += (double)v;
    dst = t;
    return CRM_OK;
  };
  if (c->working_valid) {
    st = pairs(c->cnt_f, c->n_frows, out[14]);
    if (st != CRM_OK) return st;
    st = pairs(c->cnt_m, c->n_mrows, out[15]);
    if (st != CRM_OK) return st;
  }
  return CRM_OK;
}

void crm_destroy(crm_ctx* c) { release(c); }

}  // extern "C"
