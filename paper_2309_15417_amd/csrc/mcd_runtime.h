// Host-side objects behind the C ABI (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mcd.h"
#include "mcd_internal.h"

namespace mcd {

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    ~DevBuf() { release(); }
    void release();
    mcd_status reserve(size_t need, std::string& err);                // contents not kept
    mcd_status grow_keep(size_t need, hipStream_t s, std::string& err);
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

struct MeshInfo {
    int32_t nt = 0, ntile = 0;
    int64_t tri0 = 0, tile0 = 0;
    double halo = 0, radius = 0, emax = 0;
    bool alive = false;
};

struct Particle {
    int32_t mesh = -1;
    mcd_state s{};
};

// Per-query device working set (reused by consecutive queries on a stream).
struct Workspace {
    DevBuf pairs, items, refs, part32, part64, cands, outs, pair_ub, pair_d2, pair_tie, pair_out,
        counters;
    HostBuf h_pairs, h_counters, h_pair_out;
    // time stamps
    DevBuf table, table64, eg, eg_out, pair_key, pair_t, pair_kub, ij;
    HostBuf h_key, h_t, h_ij;
};

struct Query {
    mcd_qopts opts{};
    std::vector<int32_t> pairs;          // 2n particle ids
    std::vector<PairDev> dev;
    int64_t tile_pairs_total = 0, tri_pairs_covered = 0;
    std::vector<mcd_pair_result> result;
    std::vector<mcd_contact> contacts;
    mcd_stats stats{};
    bool done = false;
};

struct Ctx {
    std::mutex mtx;
    std::string err;
    int device = 0, num_cu = 256;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t mem_budget = 0;
    int32_t n_streams = 2;
    double margin_c = 256.0;
    int32_t cand_cap = 1 << 20;
    int grid32 = 0, grid64 = 0;

    // resident triangle store
    DevBuf t32, t64, torig, tpos, trs, tsp;
    int64_t tri_cap = 0, tri_used = 0, tile_used = 0;
    std::vector<MeshInfo> meshes;
    std::unordered_map<int32_t, Particle> particles;

    Workspace ws;
    std::map<uint64_t, std::unique_ptr<Query>> tickets;
    uint64_t next_ticket = 1;

    ~Ctx()
    {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    bool hip_ok(hipError_t e, const char* what);
    TriStore store() const;
    mcd_status mesh_load(const double* xyz, int32_t nv, const int32_t* tri, int32_t nt, double eps,
                         int32_t* id);
    mcd_status particles_set(int32_t n, const int32_t* pid, const int32_t* mesh_id,
                             const mcd_state* s);
    mcd_status prepare_pairs(const int32_t* pairs, int32_t n, const mcd_qopts& o, Query& q);
    void fill_pair(PairDev& P, const Particle& A, const Particle& B, const mcd_qopts& o, double t);
    mcd_status run_static(Query& q);
    mcd_status run_toi(Query& q);
    mcd_status submit(const int32_t* pairs, int32_t n, const mcd_qopts* o, uint64_t* ticket);
    Query* find(uint64_t t);
};

}  // namespace mcd
