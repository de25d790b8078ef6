// Internal declarations shared by the HIP kernels (crm_kernels.hip) and the
// host side of the C ABI (crm_api.cpp). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace crm {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kWave = 64;        // gfx950 wavefront width
constexpr int kMaxBodies = 1024; // bodies per context
constexpr int kMaxMaterials = 256;

// Particle state as four float4 planes (structure of arrays of 16-byte
// vectors), indexed by cell-sorted slot in the working set:
//   a = (x, y, z, rho)  b = (vx, vy, vz, aux)  c = (sxx, syy, szz, sxy)
//   d = (sxz, syz, -, -)
// aux (bit pattern of b.w) = kind | body << 2 for markers, kind | material << 2
// for soil. A lane group reading the
// records of consecutive slots touches consecutive 16-byte vectors of a plane.
struct Planes {
  float4* a;
  float4* b;
  float4* c;
  float4* d;
};
struct CPlanes {
  const float4* a;
  const float4* b;
  const float4* c;
  const float4* d;
  CPlanes() = default;
  __host__ __device__ CPlanes(const Planes& p) : a(p.a), b(p.b), c(p.c), d(p.d) {}
};

enum : uint32_t { kSoilActive = 0u, kSoilExtended = 1u, kMarker = 2u };

// Rigid-body state on the device (FP64), frozen during a step.
struct Body {
  double X[3];    // origin, world
  double R[9];    // rotation body -> world, row-major
  double V[3];    // linear velocity
  double W[3];    // angular velocity (world)
  double A[3];    // linear acceleration
  double Al[3];   // angular acceleration
  double half[3]; // active box half extents (all zero: none)
  double alo[3];  // world-axis box around the box grown by 2h (a superset,
  double ahi[3];  // for a quick rejection before the exact test)
  float flo[3];   // alo, ahi rounded outwards to FP32: the same rejection
  float fhi[3];   // without FP64, exact for FP32 stored coordinates
  int32_t clo[3]; // cell indices a cell-offset position inside alo..ahi can
  int32_t chi[3]; // carry (offsets stay within one cell of [0, S))
  int32_t has_acc;
  int32_t has_box;
  int32_t place;  // pose or velocity differ from the last placement of its markers in the working set
  int32_t pad_;
};

// Cell grid of the linked list (cell size 2h) and the FP64 neighbour radius.
struct Grid {
  double lo[3];
  double inv;     // 1 / (2h), rounded once
  double R2;      // (2h)^2
  double ext;     // 2h, grow of the active boxes
  double S;       // cell size 2h
  int32_t dims[3];  // cells per axis of the grid the rebuild sorts into (a window of the domain's grid)
  int32_t org[3];   // the window's first cell in the domain's grid
  int32_t gdim[3];  // cells per axis of the domain's grid
  int32_t cell;   // positions stored as cell index + FP32 offset
  // FP32 pre-test of the list radius: an FP32 squared distance below R2lo
  // (above R2hi) is one whose FP64 value is below (above) R2; R2 (1 -+ 2^-14),
  // rounded outwards, far wider than the FP32 rounding of the distance.
  float R2lo, R2hi;
  float Sf;       // S rounded to FP32
};

// Cell-offset positions: cx is kept in d.z, cy and cz as two 16-bit signed
// halves of d.w (bit patterns of the floats), the offsets in a.xyz.
__host__ __device__ inline uint32_t pack_yz(int32_t cy, int32_t cz) {
  return (uint32_t)(uint16_t)(int16_t)cy | ((uint32_t)(uint16_t)(int16_t)cz << 16);
}
__host__ __device__ inline int32_t unpack_y(uint32_t w) { return (int32_t)(int16_t)(uint16_t)(w & 0xffffu); }
__host__ __device__ inline int32_t unpack_z(uint32_t w) { return (int32_t)(int16_t)(uint16_t)(w >> 16); }

// FP32 constants of the stage kernels.
struct Phys {
  float inv_h;
  float h;
  float kw;       // W = kw * w(q) (cubic: 1 / (pi h^3); Wendland: 21 / (16 pi h^3))
  float kf;       // grad W = kf * f(q) * (x_i - x_j) (cubic: 1 / (pi h^5); Wendland: 5 kw / h^2)
  float dt, half_dt;
  float gx, gy, gz;
  float m;        // particle mass rho0 dx^3
  float rho0;
  float two_G;    // 2G
  float iso;      // bulk_coeff K - 2G/3 (coefficient of tr(D) I)
  float av_coef;  // gamma_a h c_s m
  float xi2;      // (xi_over_h h)^2
  int32_t av_mode;
  int32_t kern;   // smoothing kernel: 0 cubic spline, 1 quintic Wendland
  float kg;       // second-derivative scale: (dF/dr) / r = kg g2(q), F = W'(r) / r
  float G;        // shear modulus, bulk factor and 1 / (2K) for the adjoint's
  float bulk;     // parameter derivatives
  float inv_2K;
  float mu_s, mu_2, I0, grain_d, cohesion, p_cri, inv_Gdt;
  int32_t cell;   // positions stored as cell index + FP32 offset
  float Sf;       // cell size 2h in FP32 (cell-offset positions)
  double S, invS; // cell size and its inverse in FP64
  double lo[3];   // grid origin
  int32_t gdim[3];  // cells per axis
  const float4* mat;  // per material: (mu_s, mu_2, cohesion, -cohesion / mu_s)
  const int32_t* bperm;  // launch order of the stage kernels' soil blocks (block_order), or null: cell order
};

// ---- static scratch of the step that allocates nothing --------------------
constexpr size_t kScratchBytes = size_t(16) << 20;  // per device, held until the process ends
constexpr int kMaxDevices = 64;
// Device address of the scratch array on `device`, which must be the current
// device; looked up on the first call per device and kept.
hipError_t scratch_address(int device, void** out);

// ---- launchers (all asynchronous on `s`) ----------------------------------

// Exclusive scan of n values into out[0..n] (out[n] = total). tmp must hold
// scan_tmp_elems(n) elements of TOut.
size_t scan_tmp_elems(int64_t n);
hipError_t scan_u32_to_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s);
hipError_t scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, hipStream_t s);

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
// dst[0] = *a, dst[1] = *b (device-side totals gathered for one read-back).
hipError_t copy2_u64(uint64_t* dst, const uint64_t* a, const uint64_t* b, hipStream_t s);
// dst[0..n) = src[0..n) (src may be mapped host memory).
hipError_t copy_f64(double* dst, const double* src, int64_t n, hipStream_t s);

// World positions x = X + R l (FP64, stored FP32 or cell + offset) of the
// markers with local indices [k0, k1) into the master planes.
hipError_t place_markers_master(const float4* local, int64_t k0, int64_t k1, int64_t n_soil, const Body* bodies,
                                Grid g, float4* m_a, float4* m_d, uint32_t* key, hipStream_t s);
// out[b], b = 0..nb: first processed-marker rank of body b (markers processed
// in id order; ids = the processed ids, NULL when all particles are processed).
hipError_t body_ranges(const int32_t* ids, int64_t n_proc, int64_t n_soil, const int64_t* bstart, int32_t nb,
                       int64_t kbase, int64_t* out, hipStream_t s);

// Activity flags of all particles (Sec. 4.2 item 2) and the count of flagged
// particles per tile of compact_counted (its first pass), into tmp.
// key: the activity pre-test's compact copy of the positions (key_words per
// particle: x, y, z FP32 bits, or the cells d.zw), kept by scatter_rows and
// place_markers_master and refilled by key_fill after whole uploads.
constexpr int key_words(bool cell) { return cell ? 2 : 3; }
hipError_t key_fill(const float4* m_a, const float4* m_d, int64_t n, bool cell, uint32_t* key, hipStream_t s);
// The union of the bodies' pre-test bounds (FP32 and cell ranges): a
// particle outside it is no candidate of any body.
struct ActUnion {
  float flo[3], fhi[3];
  int32_t clo[3], chi[3];
};
hipError_t activity_count(const float4* m_a, const float4* m_d, const uint32_t* key, int64_t n, const Body* bodies,
                          int32_t nb, const ActUnion& un, Grid g, uint8_t* flags, uint32_t* tmp, hipStream_t s);
// The same flags from an index of the master store by coarse cell (coarse_size
// list cells per axis; coarse_cells cells, their counts per axis in cd):
// ix_build lists every particle under its coarse cell (start: cells + 1
// words, fill: cells words of scratch, scan_tmp: scan_tmp_elems(cells), ids: n);
// ix_flags tests the particles listed under the coarse cells visit[0..n_visit)
// that are not marked in moved, and the first min(*n_moved, mcap) ids of
// mlist, writing their nonzero flags and counting them per compaction tile in
// bcnt (zeroed beforehand); flags_clear zeroes the flags of a list's ids;
// moved_add marks and lists (once) the ids of the rows (through slot_id) or
// the ids id0 .. id0 + n_cap - 1 (rows null).
int64_t coarse_cells(const Grid& g, int32_t cd[3]);
int32_t coarse_size();
int64_t flag_tiles(int64_t n);   // compaction tiles over n particles (bcnt words)
hipError_t ix_build(const float4* m_a, const float4* m_d, int64_t n, Grid g, uint32_t* start, uint32_t* fill,
                    uint32_t* scan_tmp, int32_t* ids, hipStream_t s);
hipError_t ix_flags(const uint32_t* visit, int64_t n_visit, const uint32_t* start, const int32_t* ids,
                    const uint8_t* moved, const int32_t* mlist, const uint64_t* n_moved, int64_t mcap,
                    const uint32_t* key, const float4* m_a, const float4* m_d, const Body* bodies, int32_t nb, Grid g,
                    uint8_t* flags, uint32_t* bcnt, hipStream_t s);
hipError_t flags_clear(const int32_t* ids, const uint64_t* n_dev, int64_t cap, uint8_t* flags, hipStream_t s);
hipError_t moved_add(const int32_t* rows, const uint64_t* n_dev, int64_t n_cap, const int32_t* slot_id, int64_t id0,
                     uint8_t* moved, int32_t* list, uint64_t* n_moved, int64_t cap, hipStream_t s);
// Order-preserving compaction of the ids with flags != 0 from those counts
// (scan, write; tiles without a flagged particle read no flag); count to
// *count_dst (device). The flag array holds flags_padded(n) bytes, zero
// beyond n; tmp holds compact_tmp_elems(n) words.
int64_t flags_padded(int64_t n);
size_t compact_tmp_elems(int64_t n);
hipError_t compact_counted(const uint8_t* flags, int64_t n, int32_t* out_ids, uint64_t* count_dst, uint32_t* tmp,
                           hipStream_t s);

// Cell hash with per-cell arrival counts (counting sort, part 1).
hipError_t hash_count(const int32_t* proc_ids, int64_t n_proc, const float4* m_a, const float4* m_d,
                      Grid g, uint32_t* key, uint32_t* rank, uint32_t* cell_cnt, hipStream_t s);
// Place into cell order with an x order key per place (part 2), then rank by
// (x, id) inside each cell and gather the master state into the sorted
// working set (part 3). tmpx holds n_proc 64-bit keys (32-bit keys in its
// first half for FP32 positions).
hipError_t place_sorted(const uint32_t* key, const uint32_t* rank, const uint32_t* cell_start,
                        int64_t n_proc, const int32_t* proc_ids, const float4* m_a, const float4* m_d, uint32_t* tmp,
                        uint64_t* tmpx, bool cell, hipStream_t s);
hipError_t gather_sorted(const uint32_t* tmp, const uint64_t* tmpx, const uint32_t* key, const int32_t* proc_ids,
                         const uint32_t* cell_start, int64_t n_proc, int64_t n_soil,
                         const uint8_t* flags, const float4* m_a, const float4* m_b,
                         const float4* m_c, const float4* m_d, Planes A, Planes B, float4* pos4,
                         int4* cpos, int32_t* slot_id, int32_t* slot_k, uint32_t* skey, bool cell,
                         hipStream_t s);

// Row lists (slots owning a neighbour list): active soil rows and marker rows.
hipError_t compact_kind(const float4* pos4, int64_t n_proc, uint32_t kind, int32_t* rows,
                        uint64_t* count_dst, uint32_t* tmp, hipStream_t s);
// Indices i < n with cnt[i] != 0, in order; count to *count_dst (device).
hipError_t compact_nonzero(const uint32_t* cnt, int64_t n, int32_t* rows, uint64_t* count_dst, uint32_t* tmp,
                           hipStream_t s);

// Neighbour lists (Alg. 1) in CSR: counts per row, offsets by an exclusive
// scan of the counts (u64, rows + 1), then the fill. A group of 8 lanes serves
// one row. soil_only keeps only soil neighbours (marker rows). The count pass
// runs over rows_cap rows with the live row count read on the device, writes
// cnt[r] = 0 beyond it, and keeps each row's first entries in `stash`
// (stash_elems(rows_cap) words), from which the fill pass copies.
size_t stash_elems(int64_t rows_cap);
hipError_t nbr_count(const int32_t* rows, int64_t rows_cap, const uint64_t* n_rows_dev,
                     const float4* pos4, const int4* cpos, const uint32_t* skey,
                     const uint32_t* cell_start, Grid g, bool soil_only, uint32_t* cnt, uint32_t* stash,
                     hipStream_t s);
// The count pass of the soil rows (not soil-only) with each block's
// candidates staged in LDS through the tile tables (tile_tables, computed for
// the same rows and device count right before it); same results as
// nbr_count. It cuts the ranges of the blocks it stages to the x interval
// their rows reach and writes the cut ranges back into tabs, so each call
// needs fresh tables.
hipError_t nbr_count_soil(const int32_t* rows, int64_t rows_cap, const uint64_t* n_rows_dev, const float4* pos4,
                          const int4* cpos, const uint32_t* skey, const uint32_t* cell_start, Grid g,
                          uint32_t* tabs, uint32_t* cnt, uint32_t* stash, hipStream_t s);
hipError_t nbr_fill(const int32_t* rows, int64_t n_rows, const float4* pos4, const int4* cpos,
                    const uint32_t* skey, const uint32_t* cell_start, Grid g, bool soil_only,
                    const uint32_t* cnt, const uint32_t* stash, const uint64_t* off, uint32_t* nbr,
                    hipStream_t s);

// Largest squared displacement of the n processed slots since the last list
// rebuild, folded into *out (float bits, integer max; *out starts at 0).
hipError_t max_disp(CPlanes A, const float4* pos4, const int4* cpos, int64_t n, bool cell, float Sf, uint32_t* out,
                    hipStream_t s);

// Per step: marker positions of the processed markers into A and B.
// cnt: the marker rows' soil-neighbour counts; rows with none also get their
// (empty-sum) BCE values here, for both states.
// all: every marker row; else only the rows of bodies whose `place` is set
// (the others keep the values of their last placement).
hipError_t place_markers_working(const int32_t* mrows, int64_t n_mrows, const uint32_t* cnt, const int32_t* slot_id,
                                 int64_t n_soil, const float4* local, const Body* bodies, Grid g, Phys P,
                                 Planes A, Planes B, bool all, hipStream_t s);

// BCE extrapolation at state S (Sec. 2.5.1); with contrib != nullptr also the
// marker accelerations and each processed marker's force and torque on its
// body (FP64, 6 per marker, at entry cidx[slot] - cbase: the marker's rank
// among the processed markers in id order).
// Rows: rows[0 .. n_near) are the marker rows that have soil neighbours
// (near_rows); the others are placed with their values by
// place_markers_working and their contrib entries stay zero.
struct NearRow {
  uint64_t k0;   // first list entry
  int32_t s;     // slot
  uint32_t n;    // entries
};
// rows[i] = (off[near[i]], mrows[near[i]], off[near[i] + 1] - off[near[i]])
// for i < n_near, once per list rebuild: the BCE passes then read one record
// per row instead of three dependent ones.
hipError_t near_rows(const int32_t* mrows, const int32_t* near, int64_t n_near, const uint64_t* off, NearRow* rows,
                     hipStream_t s);
hipError_t bce(Planes S, const NearRow* rows, int64_t n_near, const uint32_t* nbr, const Body* bodies,
               const int32_t* cidx, int64_t cbase, Phys P, double* contrib, hipStream_t s);
// Deterministic sums of 6 doubles per entry over contiguous segments: the
// plan cuts segment g = [start[g], start[g + 1]) into chunks of at most
// reduce_chunk() entries (lo/hi per chunk, first[g] = first chunk of g,
// partial = 6 per chunk); out gets 6 per segment.
struct SegPlan {
  int32_t nseg = 0;
  int64_t nchunk = 0;
  const int64_t* lo = nullptr;
  const int64_t* hi = nullptr;
  const int32_t* first = nullptr;
  double* partial = nullptr;
};
int64_t reduce_chunk();
// seq (optional, nseg counters): each segment's counter moves by one once its
// sums are written (system scope).
hipError_t segment_reduce(const double* in, const SegPlan& plan, double* out, hipStream_t s,
                          uint64_t* seq = nullptr);
// The first nb <= kBodyPack bodies uploaded to dst through a kernel's arguments.
constexpr int kBodyPack = 8;
struct BodyPack {
  Body b[kBodyPack];
};
static_assert(sizeof(BodyPack) <= 3072, "the body table fits the kernel arguments");
hipError_t put_bodies(const Body* bodies, int32_t nb, Body* dst, hipStream_t s);
// Launch order of the n_rows soil rows' blocks (kRows rows each) for the stage
// kernels, from the rows' cells in grid g: perm[p] = the block logical block p
// runs, ordered by (chunk of order_width() cells along x of the block's first
// row, its row of cells, x). cnt, first: block_order_size(g) words; base:
// that + 1; scan_tmp: scan_tmp_elems(block_order_size(g)).
int32_t order_width();
int64_t soil_block_count(int64_t rows);   // blocks of the soil rows' tile tables and stage kernels
int64_t block_order_size(const Grid& g);
hipError_t block_order(const int32_t* rows, const uint32_t* skey, int64_t n_rows, Grid g, uint32_t* cnt,
                       uint32_t* first, uint32_t* base, uint32_t* scan_tmp, int32_t* perm, hipStream_t s);

// Soil RHS + RK2 stage update (Sec. 2.2, 2.3) and, in stage 2, the return
// mapping (Sec. 2.4). With a tape, the velocity gradient of each row (and in
// stage 2 its trial stress) is also written, by slot.
struct StageTape {
  float4* l0;   // (L00, L01, L02, L10)
  float4* l1;   // (L11, L12, L20, L21)
  float4* l2;   // (L22, -, -, -)
  float4* t0;   // trial stress (sxx, syy, szz, sxy), stage 2
  float4* t1;   // (sxz, syz, -, -), stage 2
};
// tabs: the per-block tile tables of the soil rows (tile_tables, after each
// list rebuild); tix: the entries' tile positions (nbr_fill_soil).
// cfg: the LDS tile configuration (0 none, 1 small, 2 large); every
// configuration gives bit-identical results.
hipError_t fluid_stage1(CPlanes A, Planes B, const int32_t* frows, int64_t n_frows, const uint64_t* off,
                        const uint32_t* nbr, Phys P, const StageTape* tape, const uint32_t* tabs,
                        const uint16_t* tix, int cfg, hipStream_t s);
hipError_t fluid_stage2(CPlanes B, Planes A, const int32_t* frows, int64_t n_frows, const uint64_t* off,
                        const uint32_t* nbr, Phys P, const StageTape* tape, const uint32_t* tabs,
                        const uint16_t* tix, int cfg, hipStream_t s);
// Per block of soil rows: the nine slot ranges its rows' neighbours lie in
// (tile_table_words(rows_cap) words); the row count is read on the device.
// nbr_count_soil cuts the ranges of the blocks it stages.
int64_t tile_table_words(int64_t rows_cap);
hipError_t tile_tables(const int32_t* frows, int64_t rows_cap, const uint64_t* n_frows_dev, const uint32_t* skey,
                       const uint32_t* cell_start, Phys P, uint32_t* tabs, hipStream_t s);
// The fill pass of the soil rows, which also writes the tile position
// (16-bit) of each entry of the blocks the count pass staged (one per nbr
// entry; the other blocks' entries untouched); tabs from tile_tables. The
// slots of a staged block whose total is at most skip_cap are left out of
// nbr (0: every slot written); nbr_slots writes them from the positions.
hipError_t nbr_fill_soil(const int32_t* frows, int64_t n_frows, const float4* pos4, const int4* cpos,
                         const uint32_t* skey, const uint32_t* cell_start, Grid g, const uint32_t* cnt,
                         const uint32_t* stash, const uint64_t* off, uint32_t* nbr, const uint32_t* tabs,
                         uint16_t* tix, uint32_t skip_cap, hipStream_t s);
hipError_t nbr_slots(int64_t n_frows, const uint64_t* off, const uint32_t* tabs, const uint16_t* tix, uint32_t* nbr,
                     uint32_t skip_cap, hipStream_t s);
// Records of tile configuration cfg (0 for none).
uint32_t tile_records(int cfg, bool cell);

// Reverse mode (one stage at a time, see crm_adjoint.hip). Adjoint records use
// the state's plane layout: a = (x, y, z, rho), b = (u, -), c, d = stress.
hipError_t adj_local2(const int32_t* rows, int64_t n, Planes Ln, Planes Lm, Planes E, CPlanes Yn, CPlanes Ym,
                      const StageTape& T, Phys P, float* pg, hipStream_t s);
hipError_t adj_local1(const int32_t* rows, int64_t n, Planes Ln, CPlanes Lm, Planes E, CPlanes Yn,
                      const StageTape& T, Phys P, float* pg, hipStream_t s);
hipError_t adj_marker(CPlanes Y, Planes E, const int32_t* mrows, int64_t n, const uint64_t* off,
                      const uint32_t* nbr, const Body* bodies, const double* fs, Phys P, float* pg, hipStream_t s);
hipError_t adj_gather(CPlanes Y, CPlanes E, const int32_t* rows, int64_t n, const uint64_t* off,
                      const uint32_t* nbr, Phys P, Planes Lt, float* pg, hipStream_t s);
hipError_t adj_to_slots(const int32_t* rows, int64_t n, const int32_t* slot_id, CPlanes byid, Planes byslot,
                        hipStream_t s);
hipError_t adj_to_ids(const int32_t* rows, int64_t n, const int32_t* slot_id, CPlanes byslot, Planes byid,
                      hipStream_t s);
hipError_t adj_params_to_ids(int64_t n_proc, const int32_t* slot_id, float* pg, double* pid, hipStream_t s);
hipError_t adj_params_permute(int64_t n, const int32_t* perm, const double* pid, double* out, hipStream_t s);
// End-state seeds from flat device arrays (x, y, z doubles; u, stress, rho
// floats; any may be null) into id-ordered adjoint planes, and the adjoint of
// the start state back into flat arrays (*bad |= 1 on a non-finite value).
hipError_t adj_pack(int64_t n, const double* pos, const float* vel, const float* sig, const float* rho, Planes out,
                    hipStream_t s);
hipError_t adj_unpack(int64_t n, CPlanes in, double* pos, float* vel, float* sig, float* rho, uint32_t* bad,
                      hipStream_t s);

// Scatter working records back to the master planes.
hipError_t scatter_rows(CPlanes src, const int32_t* rows, int64_t n_rows, const int32_t* slot_id,
                        float4* m_a, float4* m_b, float4* m_c, float4* m_d, uint32_t* key, bool cell, hipStream_t s);
// Marker rows back to the master planes: velocity and stress (b, c, d.xy);
// the master positions stay those of the last marker placement.
hipError_t scatter_marker_rows(CPlanes src, const int32_t* rows, int64_t n_rows, const int32_t* slot_id,
                               float4* m_b, float4* m_c, float4* m_d, hipStream_t s);

}  // namespace crm
