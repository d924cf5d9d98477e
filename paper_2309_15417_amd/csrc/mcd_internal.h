// Internal layout shared by the host runtime and the gfx950 kernels.
// Not part of the public interface (include/mcd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcd.h"

namespace mcd {

constexpr int TILE = 64;   // triangles per tile; one wave holds one A tile, lane = triangle
constexpr int GROUP = 8;   // tiles per group: the coarser sphere level above the tiles

// Resident triangle store (device). Triangles of a mesh are stored in Morton
// order of their centroids, padded to a whole number of tiles. Coordinates are
// body-frame, as 9 planes of structure-of-arrays: plane k*3+c holds coordinate
// c of vertex k for every stored triangle, so a wave's 64 loads of one plane
// are one contiguous 256 B (FP32) or 512 B (FP64) segment.
struct TriStore {
    float* v32;          // 9 * cap
    double* v64;         // 9 * cap
    int32_t* orig;       // caller's face id per stored triangle (-1 for padding)
    int32_t* pos;        // per mesh region: stored index of caller's face f at tri0 + f
    float4* tile_sph;    // per tile: centre xyz, radius (rounded up), body frame
    float4* grp_sph;     // per group of GROUP consecutive tiles of a mesh: a sphere holding theirs
    float4* tri_sph;     // per triangle: centre xyz, radius (rounded up)
    float4* p32;         // per triangle, packed: 4 float4 = v0 v1 v2, unit normal, plane offset
                         // (normal and offset rounded from FP64; 3 zero)
    double2* p64;        // per triangle, packed: 5 double2 = v0 v1 v2 (9 doubles, 1 zero)
    int64_t cap;         // triangle capacity (plane stride)
};

// Per particle pair of a query (device). The relative transform takes B's body
// frame into A's body frame: X_A = M X_B + m.
struct PairDev {
    double M[9], m[3];     // FP64 relative transform
    double Ra[9], xa[3];   // A body -> world, to report points
    float Mf[9], mf[3];    // FP32 copy
    int32_t tri0_a, tri0_b;    // first stored triangle of each mesh
    int32_t na, nb;            // real triangle counts
    int32_t tile0_a, tile0_b;  // first tile of each mesh
    int32_t nta, ntb;          // tile counts
    int32_t group0_a, group0_b;  // first tile group of each mesh
    float cull;                // tile sphere gap threshold (delta + margin + motion bound)
    float thr2;                // FP32 candidate threshold (delta + mu)^2
    float thr2_np;             // same, when an edge pair is near parallel
    float mu;                  // FP32 margin
    float corr;                // lower-bound correction for near-parallel edge pairs
    double mu64, corr64;       // the same for FP64 sampling
    float vr, wa, wb;          // |v_a - v_b|, |w_a|, |w_b| (tile-level motion bound)
    double delta;              // contact threshold eps_a + eps_b
    // time stamps
    double dt, L, tol;         // step, Lipschitz bound, bisection width
    double st_a[13], st_b[13]; // states at the start of the step (x, unit q, v, w)
    int64_t table0;            // first row of the pair's FP32 sample table (12 floats per row)
    int64_t tp0;               // time stamps: first entry of the pair's tile pairs in the item list;
                               // contact sets: first word of the pair's tile-cull bitmask
    int32_t samples;           // S
    int32_t flags;
};

// What the host hands over per pair: state snapshots, the two meshes'
// records and list offsets, no arithmetic. k_pair_prep turns it into the
// PairDev record on the device (poses at time t, relative transform,
// thresholds, margins, motion bound).
struct PairSrc {
    double sa[13], sb[13];     // states at the start of the step: x, unit q (w, x, y, z), v, w
    double t;                  // pose time within the step (0: its start)
    double halo_a, halo_b;     // halo of each mesh
    double rad_a, rad_b;       // largest vertex distance from the rotation centre
    double emax_a, emax_b;     // longest edge
    int32_t tri0_a, tri0_b, na, nb, tile0_a, tile0_b, nta, ntb, group0_a, group0_b;
    int64_t table0, tp0;       // copied into PairDev
};

// Device copies of the resident particle and mesh tables, read when a pair
// list lives in device memory (the pair sources are then gathered on the
// device instead of staged by the host).
constexpr int32_t DEV_PID_LIMIT = 1 << 24;   // particle ids below this have a device record
struct PartDev {
    double s[13];              // x, unit q (w, x, y, z), v, w
    int32_t mesh;              // mesh id; -1: no particle with this id
    int32_t pad;
};
struct MeshDev {
    double halo, radius, emax;
    int32_t tri0, nt, tile0, ntile;
    int32_t alive, group0;
};
// Error bits of a device-side gather (counter word GATHER_ERR).
enum : int32_t { GATHER_BAD_ID = 1, GATHER_SAME = 2, GATHER_DEAD_MESH = 4, GATHER_OVERFLOW = 8 };

// Options shared by every pair of a query (kernel argument of k_pair_prep).
struct PrepOpts {
    double dt;                 // step (0: static query)
    double tol_rel;            // bisection width relative to dt
    double margin_c;           // FP32 margin in units of 2^-23 times the coordinate scale
    int32_t samples;
    int32_t flags;
};

// Time-stamp keys: the result of a triangle pair is a point of the dyadic
// lattice of its sample interval k (2^24 cells); key = ((k << 24) + cell) << 32
// | (caller i << 16) | caller j, so a 64-bit minimum orders by time and then by
// (i, j). A contact at the start has time part 0.
constexpr int LATTICE_BITS = 24;

// Per-wave partial counters. A counting kernel (one wave per block) writes its
// wave's count to slots[blockIdx.x] of its row instead of adding it to a
// shared counter: at the end of a persistent kernel thousands of adds to one
// address would serialise in memory. Every wave writes its slot, so rows
// need no clearing; k_stat_reduce then adds each row's first `waves` slots
// to a 64-bit counter.
constexpr int STAT_WAVES = 32768;   // slots per row (the largest grid of a counting kernel)
constexpr int STAT_ROWS = 8;
struct StatPlan {
    int32_t n;                 // rows in use
    int32_t waves[STAT_ROWS];  // grid of the kernel that wrote row i
    int32_t dst[STAT_ROWS];    // 64-bit counter (index into the counters as uint64) row i adds to
};

struct ToiOut {          // per end-game entry
    uint64_t key;
    double t;
};

struct Item {            // one (A tile, B tile) pair of one particle pair
    int32_t pair;
    int32_t tiles;       // (tile_a << 16) | tile_b, tiles local to their mesh
};

struct NearItem {        // kept tile pair of a contact-set query, with what its row test needs
    int32_t pair;
    int32_t tiles;       // (tile_a << 16) | tile_b
    int32_t a0;          // stored index of A's first triangle in the tile
    int32_t nat;         // A triangles in the tile (1..64)
    float4 cb;           // B's tile sphere centre in A's frame; radius + the near-list reach
};

struct ToiItem {         // tile pair of a time-stamp query
    int32_t pair;
    int32_t tiles;       // (tile_a << 16) | tile_b
    int32_t kfirst;      // first sample interval the tile spheres cannot exclude; -1: culled
    float dlb;           // lower bound of every triangle distance at that interval's start
};

struct ToiRec {          // triangle pair of a time-stamp query whose walk starts inside the step
    uint32_t pair;
    uint32_t ij;         // (A's stored position << 16) | B's, both local to their mesh
    int16_t kf;          // first sample interval of its tile pair
    int16_t ke;          // last sample its bounding spheres cleared (-1: none)
    float ds;            // lower bound of its distance at sample ke (or at kf when ke < 0)
};

struct NearRec {         // triangle pair whose bounding spheres are within reach
    uint32_t pt;         // pair index | 0x80000000 when the spheres overlap within mu
    uint32_t ij;         // (A's stored position << 16) | B's, both local to their mesh
};

struct Cand {            // triangle pair for the FP64 re-decision
    int32_t pair;
    int32_t ta;          // stored triangle index of A
    int32_t tb;          // stored triangle index of B
    float t;             // time stamps: start of the interval (sample index as float); static
                         // MCD_Q_VALIDATE queries: the FP32 distance estimate (see margin_tag)
};

struct PartialF {        // FP32 pass, per item
    float ub;            // min over the item of the FP32 feature distance
    float lb;            // lower bound of the item's true minimum distance
};

struct PartialD {        // FP64 pass, per item: exact lexicographic minimum
    double d2;
    int32_t ia, jb;      // caller ids
};

struct CandOut {         // FP64 result for one candidate (world frame)
    double d;
    double pa[3], pb[3];
    int32_t pair, tri_a, tri_b, keep;
    double d2;           // exact squared distance (per-pair minimum keys)
};

struct PairOut {         // per pair, written by the finalize kernel
    double d;
    double pa[3], pb[3];
    double toi;
    int32_t tri_a, tri_b, contact, status;
};

// Kernel launch entry points (mcd_kernels.hip). Counters written by one
// kernel are read by the next on the device (no host round trip); every
// consumer clamps them to the capacity of the buffer they index.
constexpr int XCD_Q_BLOCK = 8 * 16;   // int32 of one per-XCD queue set (8 counters, 64 bytes apart)

struct Launch {
    hipStream_t stream;
    int num_cu;
};

// Pair preparation: the n = hdr_src[0] records of src (n <= ncap) into
// PairDev records and the device pair count hdr_dst[0] = n. With tkey, the
// contacts at each pair's time stamp: the pose time is 0 when tkey[i] has
// time part 0, else tval[i]; a pair with tkey[i] = ~0 gets no tile pairs.
// tmode bit 1 drops both spins (translation-only motion), bit 2 maps the
// sources' tile-pair offsets to bitmask word offsets (tp0 / 64 + i, which
// leaves room for every pair's words).
constexpr int PREP_ZERO_SPIN = 1, PREP_TP0_WORDS = 2;
hipError_t launch_pair_prep(const Launch& L, const int32_t* hdr_src, const PairSrc* src, int32_t ncap,
                            const PrepOpts& o, int32_t* hdr_dst, PairDev* out, const uint64_t* tkey = nullptr,
                            const double* tval = nullptr, int tmode = 0);
// Device-side gather of pair sources from a device pair list: nlist[0] pairs
// (at most ncap) of particle ids at dlist. One PairSrc per pair from the
// particle and mesh tables, pose time t, table0 = i * rows for time stamps;
// tp0 offsets as the host staging computes them (bitmask words for contact
// sets, tile pairs for time stamps) by a one-block scan. A pair with an
// unknown id, a repeated particle or an unloaded mesh is written empty (no
// tiles) and flagged in counters[err_word]; when the totals exceed the
// capacities (tile pairs > item_cap or offset units > word_cap) every pair
// is written empty and GATHER_OVERFLOW is set. The totals go to the 64-bit
// counters c64[words_at] (offset units), c64[tiles_at] (tile pairs) and
// c64[tris_at] (triangle pairs). hdr_src[0] receives the pair count. tmp
// holds 2 * ncap int64.
hipError_t launch_pair_gather(const Launch& L, const int32_t* nlist, const int32_t* dlist, int32_t ncap,
                              const PartDev* parts, int32_t npart, const MeshDev* meshes, int32_t nmesh,
                              double t, int toi, int32_t rows, int64_t item_cap, int64_t word_cap,
                              int32_t* hdr_src, PairSrc* src, int64_t* tmp, int32_t* counters, int err_word,
                              int words_at, int tiles_at, int tris_at);
// Broad phase inside a member list of hdr[0] particle ids (at most cap),
// split into hdr[1] segments (at most seg_cap) by seg_off[0..hdr[1]] (pairs
// form inside a segment only): per member its sphere (bounding radius + halo), start centre,
// velocity and space-time box over [0, dt] (mem); pairs passing check 1
// (boxes) and check 2 (tubes) written as particle ids to pairs_out (and, if
// pos_out, as member positions), ordered by (row, column) within each
// segment; hdr_list[0] = the pair total (0 with GATHER_OVERFLOW when it
// exceeds pair_cap), c64[total_at] = the total, seg_pairs[s] = segment s's
// first pair. Unknown ids or unloaded meshes set error bits and form no pair.
struct BpMember {
    double x[3], v[3];         // centre at the start, velocity
    double r;                  // bounding radius + halo
    double lo[3], hi[3];       // space-time box over [0, dt]
    int32_t pid, end;          // particle id, end of the member's segment
    int32_t valid, pad;
};
hipError_t launch_broad_phase(const Launch& L, const int32_t* hdr, const int32_t* pid, int32_t cap,
                              const int32_t* seg_off, int32_t seg_cap, const PartDev* parts, int32_t npart,
                              const MeshDev* meshes, int32_t nmesh, double dt, BpMember* mem, int32_t* row_cnt,
                              int64_t* row_off, int64_t* seg_pairs, int32_t* hdr_list, int32_t* pairs_out,
                              int32_t* pos_out, int64_t pair_cap, int32_t* counters, int err_word, int total_at);
// Clusters: labels 0..m-1, then sweeps of min-labelling over the pairs (as
// member positions); *changed is set by a sweep that lowered a label.
hipError_t launch_label_init(const Launch& L, int32_t* label, int32_t m);
hipError_t launch_label_sweep(const Launch& L, const int32_t* pos, int64_t npairs, int32_t* label, int32_t* changed);
// Narrowing (the paper's translation-only collision-time estimate). init:
// each pair's span T = dt, no contact found yet. round (argmin 0): every
// tile pair of the items, each pair's earliest contact time in its span into
// pair_next (double bits; ~0: none); with argmin 1 the triangle pairs in
// contact at exactly T put their caller (i << 16 | j) into pair_ij. update:
// a pair with a contact records found = 1 and narrows T to an earlier
// contact, setting *changed. eval_slots: one slot row of `grid` waves (the
// triangle pairs evaluated).
hipError_t launch_narrow_init(const Launch& L, const int32_t* nq, int32_t ncap, const PairDev* pairs,
                              double* pair_T, uint64_t* pair_next, uint32_t* pair_ij, int32_t* found);
hipError_t launch_narrow_round(const Launch& L, const PairDev* pairs, const TriStore& S, const Item* items,
                               const int32_t* item_count, int64_t item_cap, const double* pair_T,
                               uint64_t* pair_next, uint32_t* pair_ij, int argmin, unsigned long long* eval_slots,
                               int grid);
hipError_t launch_narrow_update(const Launch& L, const int32_t* nq, int32_t ncap, double* pair_T,
                                uint64_t* pair_next, int32_t* found, int32_t* changed);
// Contact fusion over the sorted records of each pair (segments rec[off[p] ..
// off[p+1])): groups written in place at the start of each segment, their
// counts into ngroups (grp: one int per record, scratch); then, with goff the
// exclusive scan of ngroups, the groups gathered into out.
hipError_t launch_fuse(const Launch& L, const PairDev* pairs, const int32_t* nq, int32_t npairs, const int32_t* off,
                       mcd_contact* rec, int32_t* grp, int32_t* ngroups);
hipError_t launch_fuse_gather(const Launch& L, const int32_t* nq, int32_t npairs, const int32_t* off,
                              const int32_t* goff, const mcd_contact* rec, mcd_contact* out);
hipError_t launch_part_scatter(const Launch& L, const int32_t* ids, const PartDev* recs, int32_t n,
                               PartDev* table);

// Particle interaction (mcd_impulse.hip): one workgroup of IMP_THREADS per
// cluster (connected component of the contact graph).
constexpr int IMP_THREADS = 256;
struct ImpBody {          // a particle during the solve (world frame)
    double invm;
    double Iinv[9];       // inverse inertia about the centre of mass
    double xc[3], rc[3];  // centre of mass, and its offset from the state's origin
    double vc[3], w[3];   // velocity of the centre of mass, angular velocity
};
struct ImpContact {       // a contact in colour order: local particles, caller's index, closest points
    int32_t a, b, idx, pad;
    double pa[3], pb[3];
};
struct ImpWork {          // per contact during the solve: normal, lever arms, normal effective
    double n[3], ra[3], rb[3], kn, target;   // inverse mass, separation-speed target (fixed: orientations
    double ln, lt[3];                        // do not change), impulses
};
struct ImpOpts {
    double restitution, friction, relax, tol;
    int32_t max_iter, pad;
};
struct ImpCluster {       // a cluster's contacts [c0, c1), its ncol colour offsets from col_off[off],
    int32_t c0, c1, off, ncol;   // and its bodies [b0, b0 + nb) (contacts index them from b0)
    int32_t b0, nb;
};
constexpr int IMP_LDS_BODIES = 128;   // a cluster with at most this many bodies keeps them in LDS
hipError_t launch_impulse(const Launch& L, int32_t np, const double* state, const double* mprop, ImpBody* bodies,
                          const ImpContact* con, int32_t ncl, const ImpCluster* clusters, const int32_t* col_off,
                          const ImpOpts& o, ImpWork* work, double* impulse, const int32_t* vel_slot, double* vel,
                          int32_t* sweeps);
hipError_t launch_fill_u64(const Launch& L, uint64_t* p, int64_t n, uint64_t v);
hipError_t launch_fill_u32(const Launch& L, uint32_t* p, int64_t n, uint32_t v);
hipError_t launch_init_static(const Launch& L, uint32_t* counters, int ncounters, uint32_t* pair_ub,
                              uint64_t* pair_d2, uint64_t* pair_tie, int32_t* pair_cnt, int32_t ncap);
// nq: device pair count (read by the kernels, at most ncap). mask: one bit
// per tile pair, pair p's ceil(nta * ntb / 64) words from PairDev::tp0 on.
// Dense queries get Item records in items, contact-set queries NearItem
// records in near_items (the same buffer may serve both).
// Contact-set queries test the group spheres first and the tile pairs of the
// kept group pairs only (the kept tile pairs are those of a flat test: a
// group sphere holds its tiles' spheres); test_slots (optional): one slot
// row of cull_grid(ncap) blocks counting the sphere tests of both levels.
int cull_grid(const Launch& L, int32_t ncap);
hipError_t launch_cull(const Launch& L, const PairDev* pairs, const int32_t* nq, int32_t ncap, const TriStore& S,
                       int dense, Item* items, NearItem* near_items, int32_t* item_count, int64_t item_cap,
                       unsigned long long* tiled_count, int32_t* scan_buf, uint64_t* mask,
                       unsigned long long* test_slots = nullptr);
// bytes of scan_buf that launch_cull needs for n pairs
inline size_t cull_scan_bytes(int32_t n) { return (size_t)(2 * ((n + 1) & ~1)) * 4 + (size_t)n * 8 + 16; }
// Dense queries: every triangle pair of the items (FP32 filter with per-item
// bounds, or the exact FP64 pass with per-item lexicographic minima).
hipError_t launch_dist32(const Launch& L, const PairDev* pairs, const TriStore& S,
                         const Item* items, const int32_t* item_count, int64_t item_cap,
                         PartialF* part, uint32_t* pair_ub, Cand* cands, int32_t* cand_count,
                         int64_t cand_cap, int32_t* queue, unsigned long long* eval_slots, int grid);
hipError_t launch_dist64(const Launch& L, const PairDev* pairs, const TriStore& S,
                         const Item* items, const int32_t* item_count, int64_t item_cap,
                         PartialD* part, uint64_t* pair_d2, Cand* cands, int32_t* cand_count,
                         int64_t cand_cap, int32_t* queue, int emit_cands,
                         unsigned long long* eval_slots, int grid);
// The counting kernels below write per-wave slot rows (see StatPlan): the
// dense kernels and k_eval one row of `grid` waves, k_near two rows of
// 2 * grid waves (sphere tests; near pairs, i.e. plane-separation tests).
// k_near writes the plane-separation survivors to the near list.
hipError_t launch_near(const Launch& L, const PairDev* pairs, const TriStore& S, const NearItem* items,
                       const int32_t* item_count, int64_t item_cap, int32_t* queue, NearRec* near,
                       int32_t* near_count, int64_t near_cap, unsigned long long* test_slots,
                       unsigned long long* near_slots, int grid);
hipError_t launch_eval(const Launch& L, bool fp64, const PairDev* pairs, const TriStore& S,
                       const NearRec* near, const int32_t* near_count, int64_t near_cap, Cand* cands,
                       int32_t* cand_count, int64_t cand_cap, unsigned long long* eval_slots, int grid);
hipError_t launch_refine_select(const Launch& L, const PairDev* pairs, const Item* items,
                                const int32_t* item_count, int64_t item_cap, const PartialF* part,
                                const uint32_t* pair_ub, int dense, Item* ref_items,
                                int32_t* ref_count, int64_t ref_cap);
hipError_t launch_tie(const Launch& L, const Item* items, const int32_t* item_count,
                      int64_t item_cap, const PartialD* part, const uint64_t* pair_d2,
                      uint64_t* pair_tie);
// FP64 re-decision: one record per candidate at the candidate's index (keep
// = 0 without contact; out holds cand_cap records) and its key (pair << 32 |
// tri_a << 16 | tri_b, all ones without contact) in ckey and its squared
// distance bits in cd2 (all ones without contact); contacts per pair
// are added to pair_cnt and their total to a slot row of
// recheck_grid(cand_cap) waves. Two more rows of that size count the
// candidates within 1e-9 * delta of the threshold (band_slots) and, for
// MCD_Q_VALIDATE queries, the FP32 estimates compared (val_slots);
// ratio_max[0] receives the largest |d32 - d64| / mu over pairs without a
// near-parallel edge pair, ratio_max[1] the largest |d32 - d64| / (mu + corr)
// over pairs with one, as float bits.
int recheck_grid(int64_t cand_cap);
hipError_t launch_recheck(const Launch& L, const PairDev* pairs, const TriStore& S,
                          const Cand* cands, const int32_t* cand_count, int64_t cand_cap,
                          CandOut* out, uint64_t* ckey, uint64_t* cd2, uint64_t* pair_d2, int32_t* pair_cnt,
                          unsigned long long* kept_slots, unsigned long long* band_slots,
                          unsigned long long* val_slots, uint32_t* ratio_max);
// Contacts per pair (pair_cnt, from the re-decision) into offsets pair_off[0..n]
// (n from the device pair count nq), the largest count into max_seg[0], and
// the pairs with more than 64 contacts into large[0..max_seg[1]).
hipError_t launch_pair_scan(const Launch& L, const int32_t* nq, const int32_t* pair_cnt, int32_t* pair_off,
                            int32_t* max_seg, int32_t* large);
// Contact records sorted by (pair, tri_a, tri_b) without a global sort: the
// n re-decision keys are scattered into per-pair segments (pair_cnt is
// consumed as a cursor), and each segment of at most SEG_CAP records is
// sorted by (tri_a, tri_b) in LDS and its records gathered into `sorted`.
// seg holds n 64-bit entries; seg_p2: a power of two >= the largest segment.
constexpr int SEG_CAP = 4096;
hipError_t sort_contacts_by_pair(const Launch& L, const CandOut* out, const uint64_t* ckey, int32_t n,
                                 int32_t npairs, const int32_t* pair_off, int32_t* pair_cnt,
                                 const int32_t* large, int32_t nlarge, uint64_t* seg, int seg_p2,
                                 mcd_contact* sorted);
hipError_t launch_toi_table(const Launch& L, const PairDev* pairs, int32_t npairs, int32_t rows,
                            float* table32, double* table64);
// Space-time tile cull: one item per tile pair of every pair, at the pair's
// offset tp0 (the list holds every tile pair of the query, culled ones with
// kfirst = -1).
hipError_t launch_toi_cull(const Launch& L, const PairDev* pairs, int32_t npairs, const TriStore& S,
                           const float* table, ToiItem* items);
// Adds the per-wave slot rows of `slots` (row i at slots + i * STAT_WAVES) to
// the counters named by the plan.
hipError_t launch_stat_reduce(const Launch& L, const uint64_t* slots, const StatPlan& plan,
                              unsigned long long* counters64);
// Time-stamp sampler, stages 1 and 1b (sphere walks) and stage 2 (FP32 or
// FP64 triangle walk). queues: XCD_QUEUES counters XCD_QSTRIDE apart per
// kernel, zero at launch (2 sets for the sphere stages, 1 for the walk).
// Slot rows of `grid` waves each: the sphere stages write 4 (stage 1 gap
// evaluations, stage 1b gap evaluations, kept tile pairs, their triangle
// pairs), the walk 1 (samples), the end-game 2 (evaluations, graze leaves).
hipError_t launch_toi_spheres(const Launch& L, const PairDev* pairs, const TriStore& S, const float* table32,
                              const ToiItem* items, int64_t nitems,
                              int32_t* queues, const int32_t* pair_kub, ToiRec* trecs, int32_t* trec_count,
                              int64_t trec_cap, ToiRec* srecs, int32_t* srec_count, int64_t srec_cap,
                              unsigned long long* stat, int grid);
hipError_t launch_toi_walk(const Launch& L, const PairDev* pairs, const TriStore& S, const float* table32,
                           const double* table64, int fp64, const ToiRec* trecs, const int32_t* trec_count,
                           int64_t trec_cap, int32_t* queues, int32_t* pair_kub, Cand* eg, int32_t* eg_count,
                           int64_t eg_cap, unsigned long long* sample_slots, int grid);
hipError_t launch_toi_endgame(const Launch& L, const PairDev* pairs, const TriStore& S,
                              const Cand* eg, const int32_t* eg_count, int64_t eg_cap,
                              uint64_t* pair_key, ToiOut* out, unsigned long long* stat,
                              int from_zero, int grid);
hipError_t launch_toi_final(const Launch& L, const Cand* eg, const int32_t* eg_count,
                            int64_t eg_cap, const ToiOut* out, const uint64_t* pair_key,
                            double* pair_t);
// One given triangle pair per particle pair: (ij[2p], ij[2p + 1]), or the
// (i, j) of the pair's time-stamp key when keys is given.
hipError_t launch_pair_eval(const Launch& L, const PairDev* pairs, int32_t npairs,
                            const TriStore& S, const int32_t* ij, PairOut* out, const uint64_t* keys = nullptr);
hipError_t launch_pair_final(const Launch& L, const PairDev* pairs, const int32_t* nq, int32_t ncap,
                             const TriStore& S, const uint64_t* pair_d2, const uint64_t* pair_tie,
                             int dense, PairOut* out);
// Per pair in contact, the smallest (tri_a, tri_b) among the re-decided
// contacts at the pair's minimum (from the keys and squared distances of the
// re-decision).
hipError_t launch_tie_out(const Launch& L, const uint64_t* ckey, const uint64_t* cd2, const int32_t* count,
                          int64_t cap, const uint64_t* pair_d2, uint64_t* pair_tie);
// Contact records sorted by (pair, tri_a, tri_b) on the device: the n
// records of the re-decision (records without contact sort last), of which
// the first ncon are gathered; n and ncon are known on the host.
// temp/temp_bytes: scratch for the radix sort (query with temp = NULL).
// pair_bits / tri_bits: bits of the largest pair index and triangle index of
// the query (the radix sort runs over pair_bits + 2 tri_bits + 1 bits).
hipError_t sort_contacts(const Launch& L, const CandOut* out, int32_t n, int32_t ncon, int pair_bits,
                         int tri_bits, uint64_t* keys, uint64_t* keys_alt, int32_t* idx, int32_t* idx_alt,
                         void* temp, size_t& temp_bytes, mcd_contact* sorted);

}  // namespace mcd
