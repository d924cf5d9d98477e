// Host-side objects behind the C ABI (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <atomic>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mcd.h"
#include "mcd_internal.h"

namespace mcd {

constexpr int NCOUNTERS = 512;   // int32 device counters of a query (work queues included)
constexpr size_t PAIR_HDR = 256; // bytes before the pair records: int32 pair count, then padding
constexpr int MAX_GRAPHS = 32;   // captured chains kept per stream slot

struct Shape {                   // launch shape of the contact-set stages
    int16_t near_wpc, eval_wpc;  // waves per CU of the near-list and evaluation kernels
};

struct TuneEntry {               // autotuner state of one query bucket
    std::vector<float> ms;       // best time per shape
    int next = 0, reports = 0, best = -1;
};

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release();
    mcd_status reserve(size_t need, std::string& err);   // contents not kept
};

inline void swap(DevBuf& a, DevBuf& b) noexcept
{
    std::swap(a.p, b.p);
    std::swap(a.bytes, b.bytes);
}

// Grow-only pinned host buffer.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf() { release(); }
    void release();
    mcd_status reserve(size_t need, std::string& err);
};

// Pinned host buffers reused across queries for contact records, so the
// sorted records are copied once from the device and once to the caller.
struct PinnedPool {
    std::mutex m;
    std::vector<HostBuf*> free;
    ~PinnedPool();
    HostBuf* get(size_t bytes, std::string& err);
    void put(HostBuf* b);
};

// Device buffers reused across MCD_Q_DEVICE_OUT queries for their results.
struct DevPool {
    std::mutex m;
    std::vector<DevBuf*> free;
    ~DevPool();
    DevBuf* get(size_t bytes, std::string& err);
    void put(DevBuf* b);
};

struct MeshInfo {
    int32_t nt = 0, ntile = 0;
    int64_t tri0 = 0, tile0 = 0, group0 = 0;
    double halo = 0, radius = 0, emax = 0;
    // unit-density mass properties of the closed mesh (mass 0: it encloses
    // no volume): centre of mass and inertia tensor about it, body frame
    double mass = 0, com[3] = {0, 0, 0}, inertia[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    bool alive = false;
};

struct Particle {
    int32_t mesh = -1;
    mcd_state s{};
};

// Buffers of a device broad phase over a member list.
struct BpBufs {
    DevBuf pid, seg, mem, row_cnt, row_off, seg_pairs, pos, list, flag;
    HostBuf h_in, h_out;
};

// Device working set of one stream slot (reused by its consecutive batches).
struct Workspace {
    DevBuf pairs, items, refs, part32, part64, cands, outs, pair_ub, pair_d2, pair_tie, pair_out,
        counters;
    DevBuf src;                           // pair sources (PAIR_HDR header, then PairSrc records)
    HostBuf h_src, h_counters, h_pair_out;
    DevBuf table, table64, eg, eg_out, pair_key, pair_t, pair_kub, ij;
    HostBuf h_key, h_t, h_ij;
    DevBuf eval_out;                      // time stamps: the winning triangle pair at t* per pair
    HostBuf h_tcounters, h_eval;          // time stamps: first phase's counters, eval_out on the host
    DevBuf keys, idx, sort_tmp, sorted;   // device sort of contact records
    DevBuf near;                          // near triangle pairs (contact-set queries)
    DevBuf scan;                          // per-pair counts and offsets of the tile cull
    DevBuf trecs, srecs;                  // triangle and sphere walk lists of a time-stamp query
    DevBuf stats;                         // per-wave partial counters (STAT_ROWS rows of STAT_WAVES)
    DevBuf pair_cnt, pair_off, seg;       // contacts per pair, their offsets, per-pair segments
    DevBuf large;                         // pairs with more than 64 contacts
    DevBuf ckey, cd2;                     // re-decision keys and squared distances per candidate
    DevBuf cullmask;                      // tile-cull decisions, one bit per tile pair
    DevBuf dlist, gather_tmp;             // device pair list copy and gather scratch (device lists)
    DevBuf goff, fused;                   // contact fusion: group offsets per pair, fused records
    BpBufs bp;                            // broad phase of device cluster queries
};

// Device pair records follow a PAIR_HDR-byte header (the pair count), and
// so do the pair sources they are prepared from.
inline PairDev* pairs_dev(Workspace& ws) { return (PairDev*)((char*)ws.pairs.p + PAIR_HDR); }
inline PairSrc* src_dev(Workspace& ws) { return (PairSrc*)((char*)ws.src.p + PAIR_HDR); }

// A captured kernel chain, replayed while every argument it was captured
// with (buffer addresses, capacities, mode) is unchanged.
struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};

// A stream with its workspace and events; one worker thread drives it.
struct Slot {
    std::vector<GraphEntry> graphs;    // at most MAX_GRAPHS, least recently used replaced
    std::map<std::vector<uint64_t>, int> seen;   // time-stamp chain shapes met once (captured the second time)
    uint64_t graph_clock = 0;
    int32_t pair_cap = 0;              // capacity of the per-pair buffers (grows by 1.5x)
    int64_t item_cap = 0;              // capacity of the work-item buffers (grows by 1.5x)
    hipStream_t stream = nullptr;
    hipEvent_t ev[16] = {};            // 0-7 the static chain, 8-15 a time-stamp query's first phase
    Workspace ws;
    std::string err;
    int32_t cand_cap = 1 << 20;
    int64_t near_cap = 1 << 22;        // triangle pairs of the near list
    int64_t trec_cap = 1 << 22;        // triangle pairs of a time-stamp query's walk list
    int64_t srec_cap = 1 << 22;        // triangle pairs of its sphere walk list
    int64_t staged_tp = -1;            // tile pairs of the last time-stamp query's pairs with a time stamp
    bool hip_ok(hipError_t e, const char* what);
};

struct Query {
    mcd_qopts opts{};
    // device pair list (mcd_query_pairs_dev): read after `ready` fires on the
    // caller's stream; the pair sources are gathered on the device
    bool dev = false;
    const int32_t* d_list = nullptr;
    int32_t n_dev = 0;
    hipEvent_t ready = nullptr;
    // cluster query whose candidate pairs are found on the device: its
    // members (segments of a batch split by seg_off); n_dev is then the pair
    // capacity, and seg_pairs receives each segment's first pair
    bool cluster = false;
    std::vector<int32_t> members, seg_off;
    std::vector<int64_t> seg_pairs;
    std::vector<int32_t> pairs;        // 2n particle ids
    std::vector<MeshInfo> mi;          // 2n mesh snapshots
    std::vector<mcd_state> st;         // 2n state snapshots (unit quaternions)
    std::vector<PairSrc> src;          // per pair: snapshots and offsets for the device preparation
    int64_t tile_pairs_total = 0, tri_pairs_covered = 0, mem_estimate = 0;
    std::vector<mcd_pair_result> result;
    // contact records: pinned storage from the pool, or host storage (batch slices)
    PinnedPool* pool = nullptr;
    HostBuf* cpin = nullptr;
    std::vector<mcd_contact> cvec;
    // a query of a batch: the batch's pinned records, shared by its queries
    // (back to the pool with the last of them), from record coff on. Their
    // pair indices count from the batch's first pair; pair_base is
    // subtracted when they are copied out (mcd_fetch) or, in place, when they
    // are first viewed (mcd_result_view).
    std::shared_ptr<HostBuf> cshare;
    int64_t coff = 0;
    int32_t pair_base = 0;
    bool rebased = true;
    int64_t ncon = 0;
    mcd_contact* cdata()
    {
        return cshare ? (mcd_contact*)cshare->p + coff : (cpin ? (mcd_contact*)cpin->p : cvec.data());
    }
    // MCD_Q_DEVICE_OUT: pair results, then (at dout_con bytes) the contact
    // records, in a device buffer from the pool; dev_done fires when they are
    // written, fetched when the last mcd_fetch_dev copy out of them is done
    DevPool* dpool = nullptr;
    DevBuf* dout = nullptr;
    size_t dout_con = 0;
    hipEvent_t dev_done = nullptr, fetched = nullptr;
    ~Query()
    {
        if (cpin && pool) pool->put(cpin);
        if (ready) (void)hipEventDestroy(ready);
        if (fetched) { (void)hipEventSynchronize(fetched); (void)hipEventDestroy(fetched); }
        if (dev_done) { (void)hipEventSynchronize(dev_done); (void)hipEventDestroy(dev_done); }
        if (dout && dpool) dpool->put(dout);
    }
    // second phase of a time-stamp query (static query at each pair's t*):
    // the pair sources are the first phase's, already on the device (n_dev of
    // them); tkey / tval give each pair's time stamp (key ~0: none, the pair
    // then has no tile pairs); tmode bit 1 drops the spin (translation-only
    // narrowing), bit 2 turns tile-pair offsets into bitmask word offsets.
    // before_sync runs on the slot's stream after the chain, before the
    // query waits for it.
    bool staged = false;
    const uint64_t* tkey = nullptr;
    const double* tval = nullptr;
    int32_t tmode = 0;
    std::function<bool()> before_sync;
    int64_t grid_tile_pairs = -1;      // tile pairs that size the persistent grids and the tuning bucket (-1: all)
    int32_t npairs() const { return (dev || staged) ? n_dev : (int32_t)src.size(); }
    mcd_stats stats{};
    std::chrono::steady_clock::time_point t_submit;
    // completion
    std::mutex m;
    std::condition_variable cv;
    bool done = false;
    mcd_status status = MCD_OK;
    std::string err;
};

struct Ctx {
    PinnedPool pinned;                 // first member: outlives every query that returns buffers
    DevPool devpool;                   // as the pinned pool, for MCD_Q_DEVICE_OUT results
    std::atomic<int64_t> graph_captures{0};   // chains captured by all slots
    std::mutex mtx;                    // API calls: stores and ticket map
    std::shared_mutex store_mtx;       // device triangle store: batches share, growth excludes
    std::string err;
    int device = 0, num_cu = 256;
    hipStream_t user_stream = nullptr;
    int64_t mem_budget = 0;
    int32_t n_streams = 2;
    double margin_c = 256.0;
    int32_t cand_cap0 = 1 << 20;
    int grid32 = 0, grid64 = 0;
    bool use_graphs = true, use_tune = true;
    std::mutex tune_mtx;
    std::map<uint32_t, TuneEntry> tune;
    std::string tune_path;             // persisted autotuner table (empty: none)
    std::string device_name;
    void tune_load();
    void tune_save();
    int64_t max_batch_pairs = 1 << 16;

    // resident triangle store
    DevBuf t32, t64, torig, tpos, trs, tsp, tp32, tp64, gsp;
    int64_t tri_cap = 0, tri_used = 0, tile_cap = 0, tile_used = 0, group_cap = 0, group_used = 0;
    std::vector<MeshInfo> meshes;
    std::unordered_map<int32_t, Particle> particles;
    // device copies of the particle table (indexed by id, ids below
    // DEV_PID_LIMIT) and of the mesh table, for device-side pair gathering;
    // updated on tbl_stream. Queries that read them count as readers, and
    // every update waits until none is in flight.
    DevBuf dpart, dmesh, dstage;
    HostBuf hstage;
    int32_t dpart_cap = 0, dmesh_cap = 0;
    hipStream_t tbl_stream = nullptr;
    std::mutex rd_mtx;
    std::condition_variable rd_cv;
    int64_t dev_readers = 0;
    void wait_no_readers();
    void reader_done();
    BpBufs bp_api;                     // mcd_broad_phase (on tbl_stream)
    mcd_status upload_meshes();
    mcd_status stage_members(BpBufs& b, hipStream_t st, const std::vector<int32_t>& members,
                             const std::vector<int32_t>& seg_off, int64_t pair_cap, std::string& e);
    mcd_status broad_phase_eager(BpBufs& b, hipStream_t st, int32_t* counters, const std::vector<int32_t>& members,
                                 const std::vector<int32_t>& seg_off, double dt, DevBuf& list, bool want_pos,
                                 std::vector<int32_t>& pairs, std::vector<int64_t>& seg_pairs, std::string& e);
    mcd_status query_noalloc(int32_t n, const int32_t* d_pairs, hipStream_t st, mcd_pair_result* d_results,
                             mcd_contact* d_contacts, int64_t cap_contacts, int64_t* n_contacts);
    mcd_status impulses(int32_t n, const int32_t* pid_pairs, const mcd_contact* con, const mcd_impulse_opts* o,
                        double* impulse, int32_t* n_particles, int32_t* pids_out, double* vel_out, int32_t* sweeps);
    DevBuf imp_state, imp_mprop, imp_bodies, imp_con, imp_cl, imp_off, imp_work, imp_out, imp_vel, imp_sweeps,
        imp_slot;
    mcd_status broad_phase(int32_t n, const int32_t* pid, double dt, int32_t* cluster, int32_t* n_clusters,
                           int32_t* pairs_out, int64_t cap_pairs, int64_t* n_pairs);
    mcd_status upload_particles(int32_t n, const int32_t* pid);

    // scheduler
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<std::thread> workers;
    std::mutex qmtx;
    std::condition_variable qcv;
    std::deque<std::shared_ptr<Query>> pending;
    int64_t mem_inflight = 0;
    bool stopping = false;
    std::map<uint64_t, std::shared_ptr<Query>> tickets;
    uint64_t next_ticket = 1;

    ~Ctx();
    bool hip_ok(hipError_t e, const char* what);
    TriStore store() const;
    mcd_status start(int nslots);
    mcd_status mesh_load(const double* xyz, int32_t nv, const int32_t* tri, int32_t nt, double eps,
                         int32_t* id);
    mcd_status particles_set(int32_t n, const int32_t* pid, const int32_t* mesh_id,
                             const mcd_state* s);
    PrepOpts prep_opts(const mcd_qopts& o) const;
    mcd_status stage_src(const Query& q, Slot& s, int32_t cap, bool toi, int64_t& total);
    mcd_status check_opts(const mcd_qopts* o, mcd_qopts& out);
    mcd_status prepare_pairs(const int32_t* pairs, int32_t n, Query& q, std::string& e);
    mcd_status cluster_pairs(int32_t n, const int32_t* pid, const mcd_state* states,
                             const mcd_qopts& o, std::vector<int32_t>& out);
    mcd_status enqueue(std::shared_ptr<Query> q, uint64_t* ticket);
    std::shared_ptr<Query> find(uint64_t t);
    // execution (worker threads)
    void worker(int i);
    void run_batch(std::vector<std::shared_ptr<Query>>& batch, Slot& s);
    void run_cluster_batch(std::vector<std::shared_ptr<Query>>& batch, Slot& s);
    mcd_status run_static(Query& q, Slot& s);
    int pick_shape(uint32_t bucket, bool& measure);
    void report_shape(uint32_t bucket, int shape, float ms);
    int tune_pending(uint32_t bucket);
    mcd_status run_toi(Query& q, Slot& s);
    mcd_status run_narrow(Query& q, Slot& s, std::vector<uint64_t>& keys, std::vector<double>& times);
    bool replay(Slot& s, const std::vector<uint64_t>& key, bool capture_first, const std::function<bool()>& chain,
                bool& ran);
};

}  // namespace mcd
