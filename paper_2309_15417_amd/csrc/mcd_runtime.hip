// Host runtime behind include/mcd.h: resident mesh and particle stores,
// query preparation, a scheduler that admits queries by memory and forms
// batches, and worker threads that run each batch on their own stream
// (continuous batching: a batch is formed from whatever has arrived when a
// stream frees up, while other batches are still on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <system_error>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mcd.h"
#include "mcd_internal.h"
#include "mcd_runtime.h"

using namespace mcd;

namespace mcd {

static thread_local std::string g_create_error;
static mcd_status scratch_setup(int device, std::string& err);

// ---------------------------------------------------------------- buffers
void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

mcd_status DevBuf::reserve(size_t need, std::string& err)
{
    if (need <= bytes) return MCD_OK;
    size_t nb = std::max(need, bytes + bytes / 2);
    void* q = nullptr;
    if (hipMalloc(&q, nb) != hipSuccess) {
        (void)hipGetLastError();
        err = "device allocation of " + std::to_string(nb) + " bytes failed";
        return MCD_E_OOM;
    }
    release();
    p = q;
    bytes = nb;
    return MCD_OK;
}

void HostBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

mcd_status HostBuf::reserve(size_t need, std::string& err)
{
    if (need <= bytes) return MCD_OK;
    size_t nb = std::max(need, bytes + bytes / 2);
    void* q = nullptr;
    if (hipHostMalloc(&q, nb, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        err = "pinned host allocation of " + std::to_string(nb) + " bytes failed";
        return MCD_E_OOM;
    }
    release();
    p = q;
    bytes = nb;
    return MCD_OK;
}

PinnedPool::~PinnedPool()
{
    for (HostBuf* b : free) delete b;
}

HostBuf* PinnedPool::get(size_t bytes, std::string& err)
{
    {
        std::lock_guard<std::mutex> lk(m);
        size_t best = free.size();
        for (size_t i = 0; i < free.size(); ++i)
            if (free[i]->bytes >= bytes && (best == free.size() || free[i]->bytes < free[best]->bytes))
                best = i;
        if (best < free.size()) {
            HostBuf* b = free[best];
            free.erase(free.begin() + best);
            return b;
        }
    }
    HostBuf* b = new (std::nothrow) HostBuf();
    if (!b) { err = "host allocation failed"; return nullptr; }
    if (b->reserve(std::max<size_t>(bytes, 1 << 16), err) != MCD_OK) { delete b; return nullptr; }
    return b;
}

// Free buffers are kept up to kPinnedKeep bytes in all (the smallest freed
// first beyond that), so that a serving loop's batches find theirs again.
static constexpr size_t kPinnedKeep = (size_t)4 << 30;

void PinnedPool::put(HostBuf* b)
{
    std::lock_guard<std::mutex> lk(m);
    free.push_back(b);
    size_t held = 0;
    for (HostBuf* f : free) held += f->bytes;
    while (held > kPinnedKeep && free.size() > 1) {
        auto it = std::min_element(free.begin(), free.end(),
                                   [](HostBuf* a, HostBuf* c) { return a->bytes < c->bytes; });
        held -= (*it)->bytes;
        delete *it;
        free.erase(it);
    }
}

DevPool::~DevPool()
{
    for (DevBuf* b : free) delete b;
}

DevBuf* DevPool::get(size_t bytes, std::string& err)
{
    {
        std::lock_guard<std::mutex> lk(m);
        size_t best = free.size();
        for (size_t i = 0; i < free.size(); ++i)
            if (free[i]->bytes >= bytes && (best == free.size() || free[i]->bytes < free[best]->bytes))
                best = i;
        if (best < free.size()) {
            DevBuf* b = free[best];
            free.erase(free.begin() + best);
            return b;
        }
    }
    DevBuf* b = new (std::nothrow) DevBuf();
    if (!b) { err = "host allocation failed"; return nullptr; }
    if (b->reserve(std::max<size_t>(bytes, 1 << 16), err) != MCD_OK) { delete b; return nullptr; }
    return b;
}

void DevPool::put(DevBuf* b)
{
    std::lock_guard<std::mutex> lk(m);
    free.push_back(b);
    if (free.size() > 8) {
        auto it = std::min_element(free.begin(), free.end(),
                                   [](DevBuf* a, DevBuf* c) { return a->bytes < c->bytes; });
        delete *it;
        free.erase(it);
    }
}

// ---------------------------------------------------------------- helpers
static uint32_t spread10(uint32_t v)
{
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

static float round_up_f(double r)
{
    float f = (float)r;
    if ((double)f < r) f = std::nextafter(f, INFINITY);
    return std::nextafter(f * (1.0f + 1e-6f), INFINITY);
}

static bool hip_check(hipError_t e, const char* what, std::string& err)
{
    if (e == hipSuccess) return true;
    (void)hipGetLastError();
    err = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

bool Ctx::hip_ok(hipError_t e, const char* what) { return hip_check(e, what, err); }
bool Slot::hip_ok(hipError_t e, const char* what) { return hip_check(e, what, err); }

// ---------------------------------------------------------------- device tables
void Ctx::wait_no_readers()
{
    std::unique_lock<std::mutex> lk(rd_mtx);
    rd_cv.wait(lk, [&] { return dev_readers == 0; });
}

void Ctx::reader_done()
{
    {
        std::lock_guard<std::mutex> lk(rd_mtx);
        --dev_readers;
    }
    rd_cv.notify_all();
}

// The mesh table is small (48 B per mesh): uploaded whole after each change.
mcd_status Ctx::upload_meshes()
{
    const size_t nm = meshes.size();
    if (nm == 0) return MCD_OK;
    std::vector<MeshDev> h(nm);
    for (size_t i = 0; i < nm; ++i) {
        const MeshInfo& m = meshes[i];
        MeshDev d{};
        d.halo = m.halo; d.radius = m.radius; d.emax = m.emax;
        d.tri0 = (int32_t)m.tri0; d.nt = m.nt; d.tile0 = (int32_t)m.tile0; d.ntile = m.ntile;
        d.alive = m.alive ? 1 : 0;
        d.group0 = (int32_t)m.group0;
        h[i] = d;
    }
    mcd_status st = dmesh.reserve(nm * sizeof(MeshDev), err);
    if (st != MCD_OK) return st;
    dmesh_cap = (int32_t)(dmesh.bytes / sizeof(MeshDev));
    if (!hip_ok(hipMemcpyAsync(dmesh.p, h.data(), nm * sizeof(MeshDev), hipMemcpyHostToDevice, tbl_stream),
                "mesh table upload") ||
        !hip_ok(hipStreamSynchronize(tbl_stream), "mesh table upload"))
        return MCD_E_HIP;
    return MCD_OK;
}

// Device records of the given particles (ids below DEV_PID_LIMIT): the table
// grows to the largest id (new entries marked absent), then the records are
// staged and scattered to their ids.
mcd_status Ctx::upload_particles(int32_t n, const int32_t* pid)
{
    int32_t maxid = -1, m = 0;
    for (int i = 0; i < n; ++i)
        if (pid[i] < DEV_PID_LIMIT) { maxid = std::max(maxid, pid[i]); ++m; }
    if (m == 0) return MCD_OK;
    mcd_status st;
    if (maxid >= dpart_cap) {
        const int64_t nc = std::min<int64_t>(DEV_PID_LIMIT, std::max<int64_t>({(int64_t)maxid + 1,
                                                                               (int64_t)dpart_cap * 3 / 2, 1024}));
        DevBuf nb;
        if ((st = nb.reserve(nc * sizeof(PartDev), err)) != MCD_OK) return st;
        if (!hip_ok(hipMemsetAsync(nb.p, 0xff, nc * sizeof(PartDev), tbl_stream), "particle table") ||
            (dpart_cap > 0 && !hip_ok(hipMemcpyAsync(nb.p, dpart.p, (size_t)dpart_cap * sizeof(PartDev),
                                                     hipMemcpyDeviceToDevice, tbl_stream), "particle table")) ||
            !hip_ok(hipStreamSynchronize(tbl_stream), "particle table"))
            return MCD_E_HIP;
        mcd::swap(dpart, nb);
        dpart_cap = (int32_t)nc;
    }
    const size_t bytes = (size_t)m * (sizeof(int32_t) + sizeof(PartDev)) + 256;
    if ((st = hstage.reserve(bytes, err)) != MCD_OK || (st = dstage.reserve(bytes, err)) != MCD_OK) return st;
    PartDev* hr = (PartDev*)hstage.p;
    int32_t* hi = (int32_t*)((char*)hstage.p + (size_t)m * sizeof(PartDev));
    int k = 0;
    for (int i = 0; i < n; ++i) {
        if (pid[i] >= DEV_PID_LIMIT) continue;
        const Particle& P = particles[pid[i]];
        PartDev r{};
        std::memcpy(r.s, &P.s.x[0], sizeof r.s);
        r.mesh = P.mesh;
        hr[k] = r;
        hi[k] = pid[i];
        ++k;
    }
    PartDev* dr = (PartDev*)dstage.p;
    int32_t* di = (int32_t*)((char*)dstage.p + (size_t)m * sizeof(PartDev));
    Launch L{tbl_stream, num_cu};
    if (!hip_ok(hipMemcpyAsync(dstage.p, hstage.p, (size_t)m * (sizeof(int32_t) + sizeof(PartDev)),
                               hipMemcpyHostToDevice, tbl_stream), "particle upload") ||
        !hip_ok(launch_part_scatter(L, di, dr, m, (PartDev*)dpart.p), "particle upload") ||
        !hip_ok(hipStreamSynchronize(tbl_stream), "particle upload"))
        return MCD_E_HIP;
    return MCD_OK;
}

// ---------------------------------------------------------------- broad phase
// Member list and segment offsets to the device: the list follows a header
// (member count, segment count), as the broad-phase kernels read it.
mcd_status Ctx::stage_members(BpBufs& b, hipStream_t st, const std::vector<int32_t>& members,
                              const std::vector<int32_t>& seg_off, int64_t pair_cap, std::string& e)
{
    const size_t m = members.size(), ns = seg_off.size();   // ns = segments + 1
    mcd_status r;
    if ((r = b.pid.reserve(PAIR_HDR + sizeof(int32_t) * std::max<size_t>(m, 1), e)) != MCD_OK ||
        (r = b.seg.reserve(sizeof(int32_t) * ns, e)) != MCD_OK ||
        (r = b.mem.reserve(sizeof(BpMember) * std::max<size_t>(m, 1), e)) != MCD_OK ||
        (r = b.row_cnt.reserve(sizeof(int32_t) * std::max<size_t>(m, 1), e)) != MCD_OK ||
        (r = b.row_off.reserve(sizeof(int64_t) * std::max<size_t>(m, 1), e)) != MCD_OK ||
        (r = b.seg_pairs.reserve(sizeof(int64_t) * ns, e)) != MCD_OK ||
        (r = b.h_in.reserve(PAIR_HDR + sizeof(int32_t) * (m + ns), e)) != MCD_OK)
        return r;
    (void)pair_cap;
    int32_t* h = (int32_t*)b.h_in.p;
    std::memset(h, 0, PAIR_HDR);
    h[0] = (int32_t)m;
    h[1] = (int32_t)ns - 1;
    std::memcpy((char*)b.h_in.p + PAIR_HDR, members.data(), sizeof(int32_t) * m);
    std::memcpy((char*)b.h_in.p + PAIR_HDR + sizeof(int32_t) * m, seg_off.data(), sizeof(int32_t) * ns);
    if (!hip_check(hipMemcpyAsync(b.pid.p, b.h_in.p, PAIR_HDR + sizeof(int32_t) * m, hipMemcpyHostToDevice, st),
                   "member upload", e) ||
        !hip_check(hipMemcpyAsync(b.seg.p, (char*)b.h_in.p + PAIR_HDR + sizeof(int32_t) * m, sizeof(int32_t) * ns,
                                  hipMemcpyHostToDevice, st), "member upload", e))
        return MCD_E_HIP;
    return MCD_OK;
}

// The broad phase run eagerly on a stream, its pairs read back: `list`
// receives the header and pairs (ids), b.pos the member positions when
// want_pos. counters: 64 device int32 used for the totals and error bits.
mcd_status Ctx::broad_phase_eager(BpBufs& b, hipStream_t st, int32_t* counters, const std::vector<int32_t>& members,
                                  const std::vector<int32_t>& seg_off, double dt, DevBuf& list, bool want_pos,
                                  std::vector<int32_t>& pairs, std::vector<int64_t>& seg_pairs, std::string& e)
{
    const int32_t m = (int32_t)members.size();
    const int32_t nseg = (int32_t)seg_off.size() - 1;
    int64_t cap = std::max<int64_t>(16, 8 * (int64_t)m);
    Launch L{st, num_cu};
    for (int attempt = 0; attempt < 3; ++attempt) {
        mcd_status r;
        if ((r = stage_members(b, st, members, seg_off, cap, e)) != MCD_OK ||
            (r = list.reserve(PAIR_HDR + sizeof(int32_t) * 2 * cap, e)) != MCD_OK ||
            (want_pos && (r = b.pos.reserve(sizeof(int32_t) * 2 * cap, e)) != MCD_OK) ||
            (r = b.h_out.reserve(sizeof(int32_t) * 64 + sizeof(int64_t) * (nseg + 1), e)) != MCD_OK)
            return r;
        int32_t* hc = (int32_t*)b.h_out.p;
        if (!hip_check(hipMemsetAsync(counters, 0, 64 * sizeof(int32_t), st), "broad phase", e) ||
            !hip_check(launch_broad_phase(L, (const int32_t*)b.pid.p, (const int32_t*)((char*)b.pid.p + PAIR_HDR),
                                          std::max(m, 1), (const int32_t*)b.seg.p, std::max(nseg, 1),
                                          (const PartDev*)dpart.p, dpart_cap, (const MeshDev*)dmesh.p,
                                          (int32_t)meshes.size(), dt, (BpMember*)b.mem.p, (int32_t*)b.row_cnt.p,
                                          (int64_t*)b.row_off.p, (int64_t*)b.seg_pairs.p, (int32_t*)list.p,
                                          (int32_t*)((char*)list.p + PAIR_HDR),
                                          want_pos ? (int32_t*)b.pos.p : nullptr, cap, counters, 29, 18),
                       "broad phase", e) ||
            !hip_check(hipMemcpyAsync(hc, counters, 64 * sizeof(int32_t), hipMemcpyDeviceToHost, st), "broad phase", e) ||
            !hip_check(hipStreamSynchronize(st), "broad phase", e))
            return MCD_E_HIP;
        if (hc[29] & (GATHER_BAD_ID | GATHER_DEAD_MESH)) {
            e = (hc[29] & GATHER_BAD_ID) ? "broad phase: unknown particle id" : "broad phase: a particle uses an unloaded mesh";
            return MCD_E_NOT_FOUND;
        }
        const int64_t total = ((const int64_t*)hc)[18];
        if (total > cap) { cap = total; continue; }
        pairs.resize(2 * (size_t)total);
        seg_pairs.resize(nseg + 1);
        if ((total > 0 && !hip_check(hipMemcpyAsync(pairs.data(), (char*)list.p + PAIR_HDR,
                                                    sizeof(int32_t) * 2 * total, hipMemcpyDeviceToHost, st),
                                     "broad phase", e)) ||
            !hip_check(hipMemcpyAsync(seg_pairs.data(), b.seg_pairs.p, sizeof(int64_t) * (nseg + 1),
                                      hipMemcpyDeviceToHost, st), "broad phase", e) ||
            !hip_check(hipStreamSynchronize(st), "broad phase", e))
            return MCD_E_HIP;
        return MCD_OK;
    }
    e = "broad phase: pair list regrow did not converge";
    return MCD_E_OOM;
}

// Candidate pairs and clusters of a particle set (section 3): the broad
// phase on the device, then min-labelling sweeps over the pair graph until
// a sweep changes nothing; clusters are numbered by their first member.
// Particle interaction (section 6) for a set of contacts: the host checks the
// input, numbers the particles, colours the contact graph greedily in contact
// order (each contact takes the smallest colour that no earlier contact
// sharing one of its particles has), splits it into clusters (its connected
// components, which iterate independently) and orders the contacts by
// cluster and colour; the solve itself runs on the device, one workgroup per
// cluster.
static_assert(sizeof(mcd_state) == 13 * sizeof(double), "a state is 13 doubles: x, q, v, w");

mcd_status Ctx::impulses(int32_t n, const int32_t* pp, const mcd_contact* con, const mcd_impulse_opts* oin,
                         double* impulse, int32_t* n_particles, int32_t* pids_out, double* vel_out, int32_t* sweeps)
{
    if (n < 0 || (n > 0 && (!pp || !con))) { err = "impulses: invalid arguments"; return MCD_E_INVALID; }
    ImpOpts o{0.0, 0.0, 1.0, 1e-4, 100, 0};
    if (oin) {
        o.restitution = oin->restitution;
        o.friction = oin->friction;
        o.relax = oin->relax == 0.0 ? 1.0 : oin->relax;
        o.tol = oin->tol == 0.0 ? 1e-4 : oin->tol;
        o.max_iter = oin->max_iter == 0 ? 100 : oin->max_iter;
    }
    if (!(o.restitution >= 0.0 && o.restitution <= 1.0) || !(o.friction >= 0.0) || !std::isfinite(o.friction) ||
        !(o.relax > 0.0 && o.relax <= 1.0) || !(o.tol > 0.0) || !std::isfinite(o.tol) || o.max_iter < 1 ||
        o.max_iter > 1000000) {
        err = "impulses: restitution in [0, 1], friction >= 0, relax in (0, 1], tol > 0, 1 <= max_iter <= 1e6";
        return MCD_E_INVALID;
    }
    // particles in order of first appearance
    std::unordered_map<int32_t, int32_t> local;
    std::vector<int32_t> pids;
    std::vector<int32_t> ab(2 * (size_t)n);
    for (int32_t k = 0; k < 2 * n; ++k) {
        const int32_t id = pp[k];
        auto it = local.find(id);
        if (it == local.end()) {
            auto pt = particles.find(id);
            if (pt == particles.end()) { err = "impulses: unknown particle id " + std::to_string(id); return MCD_E_NOT_FOUND; }
            const int32_t m = pt->second.mesh;
            if (m < 0 || m >= (int32_t)meshes.size() || !meshes[m].alive || !(meshes[m].mass > 0.0)) {
                err = "impulses: particle " + std::to_string(id) + " has no mesh enclosing a volume";
                return MCD_E_INVALID;
            }
            it = local.emplace(id, (int32_t)pids.size()).first;
            pids.push_back(id);
        }
        ab[k] = it->second;
    }
    for (int32_t c = 0; c < n; ++c)
        if (ab[2 * c] == ab[2 * c + 1]) { err = "impulses: a contact joins a particle to itself"; return MCD_E_INVALID; }
    const int32_t np = (int32_t)pids.size();
    if (n_particles) *n_particles = np;
    if (pids_out && np) std::memcpy(pids_out, pids.data(), sizeof(int32_t) * np);
    if (n == 0) {
        if (sweeps) *sweeps = 0;
        return MCD_OK;
    }
    // greedy colouring in contact order
    std::vector<std::vector<int32_t>> used(np);
    std::vector<int32_t> col(n);
    int32_t ncol = 0;
    for (int32_t c = 0; c < n; ++c) {
        const auto &ua = used[ab[2 * c]], &ub = used[ab[2 * c + 1]];
        int32_t k = 0;
        while (std::find(ua.begin(), ua.end(), k) != ua.end() || std::find(ub.begin(), ub.end(), k) != ub.end()) ++k;
        col[c] = k;
        used[ab[2 * c]].push_back(k);
        used[ab[2 * c + 1]].push_back(k);
        ncol = std::max(ncol, k + 1);
    }
    // clusters: connected components of the contact graph (union-find),
    // numbered in order of their first contact
    std::vector<int32_t> up(np);
    for (int32_t i = 0; i < np; ++i) up[i] = i;
    auto root = [&](int32_t x) {
        while (up[x] != x) x = up[x] = up[up[x]];
        return x;
    };
    for (int32_t c = 0; c < n; ++c) {
        const int32_t x = root(ab[2 * c]), y = root(ab[2 * c + 1]);
        if (x != y) up[std::max(x, y)] = std::min(x, y);
    }
    std::vector<int32_t> cl_of_root(np, -1), cl(n);
    int32_t ncl = 0;
    for (int32_t c = 0; c < n; ++c) {
        int32_t& k = cl_of_root[root(ab[2 * c])];
        if (k < 0) k = ncl++;
        cl[c] = k;
    }
    // contacts ordered by (cluster, colour, index); per cluster its range and
    // colour offsets
    std::vector<int32_t> order(n);
    for (int32_t c = 0; c < n; ++c) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return std::make_tuple(cl[x], col[x], x) < std::make_tuple(cl[y], col[y], y);
    });
    // bodies renumbered cluster by cluster (in order of first appearance
    // within each); slot: a body's place in the caller's particle order
    std::vector<ImpCluster> hcl(ncl);
    std::vector<int32_t> cl_of_body(np), nb(ncl, 0), newidx(np), slot(np);
    for (int32_t i = 0; i < np; ++i) {
        cl_of_body[i] = cl_of_root[root(i)];
        ++nb[cl_of_body[i]];
    }
    for (int32_t k = 0, b0 = 0; k < ncl; ++k) {
        hcl[k].b0 = b0;
        hcl[k].nb = nb[k];
        b0 += nb[k];
    }
    {
        std::vector<int32_t> fill(ncl);
        for (int32_t k = 0; k < ncl; ++k) fill[k] = hcl[k].b0;
        for (int32_t i = 0; i < np; ++i) {
            newidx[i] = fill[cl_of_body[i]]++;
            slot[newidx[i]] = i;
        }
    }
    std::vector<int32_t> off;
    std::vector<ImpContact> hc(n);
    for (int32_t r = 0; r < n;) {
        const int32_t k = cl[order[r]];
        ImpCluster& g = hcl[k];
        g.c0 = r;
        g.off = (int32_t)off.size();
        int32_t last = -1;
        for (; r < n && cl[order[r]] == k; ++r) {
            const int32_t c = order[r];
            while (last < col[c]) { off.push_back(r); ++last; }
            ImpContact& rc = hc[r];
            rc.a = newidx[ab[2 * c]] - g.b0;
            rc.b = newidx[ab[2 * c + 1]] - g.b0;
            rc.idx = c;
            rc.pad = 0;
            for (int i = 0; i < 3; ++i) { rc.pa[i] = con[c].pa[i]; rc.pb[i] = con[c].pb[i]; }
        }
        g.c1 = r;
        g.ncol = last + 1;
        off.push_back(r);
    }
    std::vector<double> hs(13 * (size_t)np), hm(13 * (size_t)np);
    for (int32_t j = 0; j < np; ++j) {   // in the cluster-by-cluster order
        const Particle& P = particles.at(pids[slot[j]]);
        std::memcpy(&hs[13 * (size_t)j], &P.s, sizeof(double) * 13);
        const MeshInfo& mi = meshes[P.mesh];
        hm[13 * (size_t)j] = mi.mass;
        std::memcpy(&hm[13 * (size_t)j + 1], mi.com, sizeof(double) * 3);
        std::memcpy(&hm[13 * (size_t)j + 4], mi.inertia, sizeof(double) * 9);
    }
    mcd_status st;
    if ((st = imp_state.reserve(sizeof(double) * hs.size(), err)) != MCD_OK ||
        (st = imp_mprop.reserve(sizeof(double) * hm.size(), err)) != MCD_OK ||
        (st = imp_bodies.reserve(sizeof(ImpBody) * np, err)) != MCD_OK ||
        (st = imp_con.reserve(sizeof(ImpContact) * n, err)) != MCD_OK ||
        (st = imp_cl.reserve(sizeof(ImpCluster) * ncl, err)) != MCD_OK ||
        (st = imp_off.reserve(sizeof(int32_t) * off.size(), err)) != MCD_OK ||
        (st = imp_work.reserve(sizeof(ImpWork) * n, err)) != MCD_OK ||
        (st = imp_out.reserve(sizeof(double) * 4 * n, err)) != MCD_OK ||
        (st = imp_vel.reserve(sizeof(double) * 6 * np, err)) != MCD_OK ||
        (st = imp_sweeps.reserve(sizeof(int32_t) * ncl, err)) != MCD_OK ||
        (st = imp_slot.reserve(sizeof(int32_t) * np, err)) != MCD_OK)
        return st;
    hipStream_t sm = user_stream;
    Launch L{sm, num_cu};
    std::vector<double> himp(4 * (size_t)n), hvel(6 * (size_t)np);
    std::vector<int32_t> hsw(ncl);
    if (!hip_ok(hipSetDevice(device), "impulses") ||
        !hip_ok(hipMemcpyAsync(imp_state.p, hs.data(), sizeof(double) * hs.size(), hipMemcpyHostToDevice, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(imp_mprop.p, hm.data(), sizeof(double) * hm.size(), hipMemcpyHostToDevice, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(imp_con.p, hc.data(), sizeof(ImpContact) * n, hipMemcpyHostToDevice, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(imp_cl.p, hcl.data(), sizeof(ImpCluster) * ncl, hipMemcpyHostToDevice, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(imp_off.p, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(imp_slot.p, slot.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, sm), "impulses") ||
        !hip_ok(launch_impulse(L, np, (const double*)imp_state.p, (const double*)imp_mprop.p, (ImpBody*)imp_bodies.p,
                               (const ImpContact*)imp_con.p, ncl, (const ImpCluster*)imp_cl.p,
                               (const int32_t*)imp_off.p, o, (ImpWork*)imp_work.p, (double*)imp_out.p,
                               (const int32_t*)imp_slot.p, (double*)imp_vel.p, (int32_t*)imp_sweeps.p), "impulses") ||
        !hip_ok(hipMemcpyAsync(himp.data(), imp_out.p, sizeof(double) * himp.size(), hipMemcpyDeviceToHost, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(hvel.data(), imp_vel.p, sizeof(double) * hvel.size(), hipMemcpyDeviceToHost, sm), "impulses") ||
        !hip_ok(hipMemcpyAsync(hsw.data(), imp_sweeps.p, sizeof(int32_t) * ncl, hipMemcpyDeviceToHost, sm), "impulses") ||
        !hip_ok(hipStreamSynchronize(sm), "impulses"))
        return MCD_E_HIP;
    if (impulse) std::memcpy(impulse, himp.data(), sizeof(double) * himp.size());
    if (vel_out) std::memcpy(vel_out, hvel.data(), sizeof(double) * hvel.size());
    if (sweeps) *sweeps = *std::max_element(hsw.begin(), hsw.end());
    return MCD_OK;
}

mcd_status Ctx::broad_phase(int32_t n, const int32_t* pid, double dt, int32_t* cluster, int32_t* n_clusters,
                            int32_t* pairs_out, int64_t cap_pairs, int64_t* n_pairs)
{
    if (n < 0 || (n > 0 && !pid) || !(dt >= 0.0) || !std::isfinite(dt)) {
        err = "broad_phase: invalid arguments";
        return MCD_E_INVALID;
    }
    {
        std::vector<int32_t> ids(pid, pid + n);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end()) { err = "broad_phase: particle listed twice"; return MCD_E_INVALID; }
        for (int i = 0; i < n; ++i)
            if (pid[i] < 0 || pid[i] >= DEV_PID_LIMIT || particles.find(pid[i]) == particles.end()) {
                err = "broad_phase: unknown particle id " + std::to_string(pid[i]) + " (ids must be below 2^24)";
                return MCD_E_NOT_FOUND;
            }
    }
    std::vector<int32_t> members(pid, pid + n), seg_off = {0, n}, pairs;
    std::vector<int64_t> seg_pairs;
    mcd_status st;
    if ((st = bp_api.flag.reserve(sizeof(int32_t) * 64, err)) != MCD_OK) return st;
    int32_t* cnt = (int32_t*)bp_api.flag.p;
    DevBuf& list = bp_api.list;
    if ((st = broad_phase_eager(bp_api, tbl_stream, cnt, members, seg_off, dt, list, true, pairs, seg_pairs, err)) !=
        MCD_OK)
        return st;
    const int64_t np = (int64_t)pairs.size() / 2;
    if (n_pairs) *n_pairs = np;
    if (pairs_out && np > cap_pairs) { err = "broad_phase: pair capacity too small"; return MCD_E_INVALID; }
    if (pairs_out && np > 0) std::memcpy(pairs_out, pairs.data(), sizeof(int32_t) * 2 * np);
    if (cluster || n_clusters) {
        DevBuf lab;
        if ((st = lab.reserve(sizeof(int32_t) * std::max(n, 1), err)) != MCD_OK) return st;
        Launch L{tbl_stream, num_cu};
        if (!hip_ok(launch_label_init(L, (int32_t*)lab.p, n), "clusters")) return MCD_E_HIP;
        int32_t* hflag = (int32_t*)bp_api.h_out.p;
        for (int round = 0;; ++round) {
            // four sweeps per check of the flag
            bool ok = hip_ok(hipMemsetAsync(cnt, 0, sizeof(int32_t), tbl_stream), "clusters");
            for (int k = 0; ok && k < 4; ++k)
                ok = hip_ok(launch_label_sweep(L, (const int32_t*)bp_api.pos.p, np, (int32_t*)lab.p, cnt), "clusters");
            ok = ok && hip_ok(hipMemcpyAsync(hflag, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, tbl_stream), "clusters") &&
                 hip_ok(hipStreamSynchronize(tbl_stream), "clusters");
            if (!ok) return MCD_E_HIP;
            if (hflag[0] == 0) break;
            if (round > n) { err = "clusters: labelling did not converge"; return MCD_E_INVALID; }
        }
        std::vector<int32_t> label(n);
        if (n > 0 && (!hip_ok(hipMemcpy(label.data(), lab.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost), "clusters")))
            return MCD_E_HIP;
        // a component's label is its first member's position: number the
        // clusters in that order
        std::vector<int32_t> id(n, -1);
        int32_t k = 0;
        for (int i = 0; i < n; ++i) {
            const int32_t l = label[i];
            if (id[l] < 0) id[l] = k++;
            if (cluster) cluster[i] = id[l];
        }
        if (n_clusters) *n_clusters = k;
    }
    return MCD_OK;
}

// ---------------------------------------------------------------- meshes
// Unit-density mass properties of a closed triangle mesh (the masses of the
// particle interaction, section 6), by the divergence theorem: each face with
// the origin spans a signed tetrahedron of volume a.(b x c)/6, first moment
// vol (a+b+c)/4 and second moment vol/20 (aa' + bb' + cc' + ss'), s = a+b+c.
// Inward-facing meshes come out negative and are flipped; a mesh that
// encloses no volume gets mass 0.
static void mass_properties(const double* xyz, const int32_t* tri, int32_t nt, MeshInfo& mi)
{
    double vol = 0.0, mom[3] = {0.0, 0.0, 0.0}, sec[9] = {0.0};
    for (int32_t f = 0; f < nt; ++f) {
        const double* a = xyz + 3 * tri[3 * f];
        const double* b = xyz + 3 * tri[3 * f + 1];
        const double* c = xyz + 3 * tri[3 * f + 2];
        const double bxc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
        const double v = (a[0] * bxc[0] + a[1] * bxc[1] + a[2] * bxc[2]) / 6.0;
        const double sum[3] = {a[0] + b[0] + c[0], a[1] + b[1] + c[1], a[2] + b[2] + c[2]};
        vol += v;
        for (int i = 0; i < 3; ++i) mom[i] += v * sum[i] / 4.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                sec[3 * i + j] += v / 20.0 * (a[i] * a[j] + b[i] * b[j] + c[i] * c[j] + sum[i] * sum[j]);
    }
    const double sg = vol < 0.0 ? -1.0 : 1.0;
    vol *= sg;
    if (!(vol > 0.0) || !std::isfinite(vol)) { mi.mass = 0.0; return; }
    double cm[3];
    for (int i = 0; i < 3; ++i) cm[i] = sg * mom[i] / vol;
    const double trace = sg * (sec[0] + sec[4] + sec[8]);
    const double c2 = cm[0] * cm[0] + cm[1] * cm[1] + cm[2] * cm[2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double about_origin = (i == j ? trace : 0.0) - sg * sec[3 * i + j];
            mi.inertia[3 * i + j] = about_origin - vol * ((i == j ? c2 : 0.0) - cm[i] * cm[j]);
        }
    mi.mass = vol;
    for (int i = 0; i < 3; ++i) mi.com[i] = cm[i];
}

mcd_status Ctx::mesh_load(const double* xyz, int32_t nv, const int32_t* tri, int32_t nt, double eps,
                          int32_t* id)
{
    if (!xyz || !tri || !id || nv < 3 || nt < 1 || nt > 65535 || !(eps >= 0.0) ||
        !std::isfinite(eps)) {
        err = "mesh_load: invalid arguments (need nv >= 3, 1 <= nt <= 65535, finite eps >= 0)";
        return MCD_E_INVALID;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < 3 * (int64_t)nv; ++i)
        if (!std::isfinite(xyz[i])) { err = "mesh_load: non-finite vertex coordinate"; return MCD_E_INVALID; }
    for (int i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], xyz[3 * i + c]);
            hi[c] = std::max(hi[c], xyz[3 * i + c]);
        }
    double diag2 = 0;
    for (int c = 0; c < 3; ++c) diag2 += (hi[c] - lo[c]) * (hi[c] - lo[c]);
    for (int64_t f = 0; f < nt; ++f) {
        int a = tri[3 * f], b = tri[3 * f + 1], c = tri[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) {
            err = "mesh_load: vertex index out of range in face " + std::to_string(f);
            return MCD_E_INVALID;
        }
        const double *p = xyz + 3 * a, *q = xyz + 3 * b, *r = xyz + 3 * c;
        double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        double v[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
        double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        double area = 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(area > 1e-14 * diag2)) {
            err = "mesh_load: zero-area face " + std::to_string(f);
            return MCD_E_INVALID;
        }
    }
    // Morton order of centroids within the mesh's bounding box.
    std::vector<std::pair<uint32_t, int32_t>> key(nt);
    for (int f = 0; f < nt; ++f) {
        uint32_t k = 0;
        uint32_t qv[3];
        for (int c = 0; c < 3; ++c) {
            double m = (xyz[3 * tri[3 * f] + c] + xyz[3 * tri[3 * f + 1] + c] + xyz[3 * tri[3 * f + 2] + c]) / 3.0;
            double s = hi[c] > lo[c] ? (m - lo[c]) / (hi[c] - lo[c]) : 0.0;
            qv[c] = (uint32_t)std::min(1023.0, std::max(0.0, s * 1023.0));
        }
        k = spread10(qv[0]) | (spread10(qv[1]) << 1) | (spread10(qv[2]) << 2);
        key[f] = {k, f};
    }
    std::sort(key.begin(), key.end());
    const int ntile = (nt + TILE - 1) / TILE;
    const int npad = ntile * TILE;

    MeshInfo mi;
    mi.nt = nt;
    mi.ntile = ntile;
    mi.halo = eps;
    mi.tri0 = tri_used;
    mi.tile0 = tile_used;
    double R = 0, emax = 0;
    for (int i = 0; i < nv; ++i)
        R = std::max(R, std::sqrt(xyz[3 * i] * xyz[3 * i] + xyz[3 * i + 1] * xyz[3 * i + 1] +
                                  xyz[3 * i + 2] * xyz[3 * i + 2]));
    mi.radius = R;
    mass_properties(xyz, tri, nt, mi);

    // Host staging of the new region.
    std::vector<float> v32(9 * (size_t)npad);
    std::vector<double> v64(9 * (size_t)npad);
    std::vector<int32_t> orig(npad, -1), pos(npad, 0);
    std::vector<float4> tsph(ntile), trsph(npad);
    std::vector<float4> pk32(4 * (size_t)npad);    // packed copies for per-lane gathers
    std::vector<double2> pk64(5 * (size_t)npad);
    for (int s = 0; s < npad; ++s) {
        int f = key[std::min(s, nt - 1)].second;
        if (s < nt) { orig[s] = f; pos[f] = mi.tri0 + s; }
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) {
                double x = xyz[3 * tri[3 * f + k] + c];
                v64[(size_t)(3 * k + c) * npad + s] = x;
                v32[(size_t)(3 * k + c) * npad + s] = (float)x;
            }
        for (int k = 0; k < 3; ++k) {
            const double* p = xyz + 3 * tri[3 * f + k];
            const double* q = xyz + 3 * tri[3 * f + (k + 1) % 3];
            double e2 = (p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) + (p[2] - q[2]) * (p[2] - q[2]);
            emax = std::max(emax, std::sqrt(e2));
        }
    }
    mi.emax = emax;
    for (int t = 0; t < npad; ++t) {
        float f[12] = {0};
        double g[10] = {0};
        for (int k = 0; k < 9; ++k) {
            f[k] = v32[(size_t)k * npad + t];
            g[k] = v64[(size_t)k * npad + t];
        }
        // plane of the triangle (unit normal, offset) from the FP64 vertices
        const double u[3] = {g[3] - g[0], g[4] - g[1], g[5] - g[2]}, w[3] = {g[6] - g[0], g[7] - g[1], g[8] - g[2]};
        double nn[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const double nl = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        for (int c = 0; c < 3; ++c) nn[c] /= nl;
        const double off = nn[0] * g[0] + nn[1] * g[1] + nn[2] * g[2];
        pk32[4 * (size_t)t + 0] = make_float4(f[0], f[1], f[2], f[3]);
        pk32[4 * (size_t)t + 1] = make_float4(f[4], f[5], f[6], f[7]);
        pk32[4 * (size_t)t + 2] = make_float4(f[8], (float)nn[0], (float)nn[1], (float)nn[2]);
        pk32[4 * (size_t)t + 3] = make_float4((float)off, 0.f, 0.f, 0.f);
        for (int q = 0; q < 5; ++q) pk64[5 * (size_t)t + q] = make_double2(g[2 * q], g[2 * q + 1]);
    }
    // Bounding spheres of the FP32 vertices (tile and triangle), radius rounded up.
    auto sphere = [&](int s0, int s1) {
        double lo2[3] = {INFINITY, INFINITY, INFINITY}, hi2[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int s = s0; s < s1; ++s)
            for (int k = 0; k < 3; ++k)
                for (int c = 0; c < 3; ++c) {
                    double x = v32[(size_t)(3 * k + c) * npad + s];
                    lo2[c] = std::min(lo2[c], x);
                    hi2[c] = std::max(hi2[c], x);
                }
        float cx = (float)(0.5 * (lo2[0] + hi2[0])), cy = (float)(0.5 * (lo2[1] + hi2[1])),
              cz = (float)(0.5 * (lo2[2] + hi2[2]));
        double r = 0;
        for (int s = s0; s < s1; ++s)
            for (int k = 0; k < 3; ++k) {
                double dx = v32[(size_t)(3 * k) * npad + s] - (double)cx;
                double dy = v32[(size_t)(3 * k + 1) * npad + s] - (double)cy;
                double dz = v32[(size_t)(3 * k + 2) * npad + s] - (double)cz;
                r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
        return make_float4(cx, cy, cz, round_up_f(r));
    };
    for (int t = 0; t < ntile; ++t) tsph[t] = sphere(t * TILE, std::min(nt, (t + 1) * TILE));
    // Group spheres (the coarser level): GROUP consecutive tiles (Morton
    // order keeps them close), a sphere about the box of their spheres that
    // holds each of them, computed in FP64 and rounded up.
    const int ngroup = (ntile + GROUP - 1) / GROUP;
    std::vector<float4> gsph(ngroup);
    for (int g = 0; g < ngroup; ++g) {
        const int t0 = g * GROUP, t1 = std::min(ntile, t0 + GROUP);
        double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int t = t0; t < t1; ++t) {
            const double c[3] = {tsph[t].x, tsph[t].y, tsph[t].z};
            for (int k = 0; k < 3; ++k) {
                lo3[k] = std::min(lo3[k], c[k] - tsph[t].w);
                hi3[k] = std::max(hi3[k], c[k] + tsph[t].w);
            }
        }
        const float cx = (float)(0.5 * (lo3[0] + hi3[0])), cy = (float)(0.5 * (lo3[1] + hi3[1])),
                    cz = (float)(0.5 * (lo3[2] + hi3[2]));
        double r = 0.0;
        for (int t = t0; t < t1; ++t) {
            const double dx = tsph[t].x - (double)cx, dy = tsph[t].y - (double)cy, dz = tsph[t].z - (double)cz;
            r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz) + (double)tsph[t].w);
        }
        gsph[g] = make_float4(cx, cy, cz, round_up_f(r));
    }
    for (int s = 0; s < npad; ++s) trsph[s] = sphere(std::min(s, nt - 1), std::min(s, nt - 1) + 1);

    // Device store: grow (keeping contents) and append. Growth replaces the
    // buffers, so it waits for running batches (exclusive store lock), and
    // the mesh table changes, so it waits for device-list queries.
    wait_no_readers();
    std::unique_lock<std::shared_mutex> lk(store_mtx);
    const int64_t need_tri = tri_used + npad;
    if (need_tri > tri_cap) {
        int64_t nc = std::max<int64_t>(need_tri, std::max<int64_t>(1 << 16, tri_cap * 2));
        // Planes are strided by the capacity: re-layout into new buffers.
        DevBuf n32, n64, norig, npos, ntrs, np32, np64;
        mcd_status st;
        if ((st = np32.reserve(4 * nc * sizeof(float4), err)) != MCD_OK) return st;
        if ((st = np64.reserve(5 * nc * sizeof(double2), err)) != MCD_OK) return st;
        if ((st = n32.reserve(9 * nc * sizeof(float), err)) != MCD_OK) return st;
        if ((st = n64.reserve(9 * nc * sizeof(double), err)) != MCD_OK) return st;
        if ((st = norig.reserve(nc * sizeof(int32_t), err)) != MCD_OK) return st;
        if ((st = npos.reserve(nc * sizeof(int32_t), err)) != MCD_OK) return st;
        if ((st = ntrs.reserve(nc * sizeof(float4), err)) != MCD_OK) return st;
        if (tri_used > 0) {
            for (int k = 0; k < 9; ++k) {
                if (!hip_ok(hipMemcpy((float*)n32.p + k * nc, (float*)t32.p + k * tri_cap,
                                      tri_used * sizeof(float), hipMemcpyDeviceToDevice), "store copy") ||
                    !hip_ok(hipMemcpy((double*)n64.p + k * nc, (double*)t64.p + k * tri_cap,
                                      tri_used * sizeof(double), hipMemcpyDeviceToDevice), "store copy"))
                    return MCD_E_HIP;
            }
            if (!hip_ok(hipMemcpy(norig.p, torig.p, tri_used * 4, hipMemcpyDeviceToDevice), "store copy") ||
                !hip_ok(hipMemcpy(npos.p, tpos.p, tri_used * 4, hipMemcpyDeviceToDevice), "store copy") ||
                !hip_ok(hipMemcpy(ntrs.p, trs.p, tri_used * sizeof(float4), hipMemcpyDeviceToDevice), "store copy") ||
                !hip_ok(hipMemcpy(np32.p, tp32.p, 4 * tri_used * sizeof(float4), hipMemcpyDeviceToDevice), "store copy") ||
                !hip_ok(hipMemcpy(np64.p, tp64.p, 5 * tri_used * sizeof(double2), hipMemcpyDeviceToDevice), "store copy"))
                return MCD_E_HIP;
        }
        mcd::swap(t32, n32); mcd::swap(t64, n64); mcd::swap(torig, norig); mcd::swap(tpos, npos);
        mcd::swap(trs, ntrs); mcd::swap(tp32, np32); mcd::swap(tp64, np64);
        tri_cap = nc;
    }
    if (tile_used + ntile > tile_cap) {
        int64_t nc = std::max<int64_t>(tile_used + ntile, std::max<int64_t>(1 << 12, tile_cap * 2));
        DevBuf nt_;
        mcd_status st = nt_.reserve(nc * sizeof(float4), err);
        if (st != MCD_OK) return st;
        if (tile_used > 0 &&
            !hip_ok(hipMemcpy(nt_.p, tsp.p, tile_used * sizeof(float4), hipMemcpyDeviceToDevice), "store copy"))
            return MCD_E_HIP;
        mcd::swap(tsp, nt_);
        tile_cap = nc;
    }
    if (group_used + ngroup > group_cap) {
        int64_t nc = std::max<int64_t>(group_used + ngroup, std::max<int64_t>(1 << 10, group_cap * 2));
        DevBuf ng_;
        mcd_status st = ng_.reserve(nc * sizeof(float4), err);
        if (st != MCD_OK) return st;
        if (group_used > 0 &&
            !hip_ok(hipMemcpy(ng_.p, gsp.p, group_used * sizeof(float4), hipMemcpyDeviceToDevice), "store copy"))
            return MCD_E_HIP;
        mcd::swap(gsp, ng_);
        group_cap = nc;
    }
    if (!hip_ok(hipMemcpy((float4*)gsp.p + group_used, gsph.data(), ngroup * sizeof(float4), hipMemcpyHostToDevice),
                "mesh upload"))
        return MCD_E_HIP;
    mi.group0 = group_used;
    group_used += ngroup;
    for (int k = 0; k < 9; ++k) {
        if (!hip_ok(hipMemcpy((float*)t32.p + k * tri_cap + tri_used, v32.data() + (size_t)k * npad,
                              npad * sizeof(float), hipMemcpyHostToDevice), "mesh upload") ||
            !hip_ok(hipMemcpy((double*)t64.p + k * tri_cap + tri_used, v64.data() + (size_t)k * npad,
                              npad * sizeof(double), hipMemcpyHostToDevice), "mesh upload"))
            return MCD_E_HIP;
    }
    if (!hip_ok(hipMemcpy((int32_t*)torig.p + tri_used, orig.data(), npad * 4, hipMemcpyHostToDevice), "mesh upload") ||
        !hip_ok(hipMemcpy((int32_t*)tpos.p + tri_used, pos.data(), npad * 4, hipMemcpyHostToDevice), "mesh upload") ||
        !hip_ok(hipMemcpy((float4*)trs.p + tri_used, trsph.data(), npad * sizeof(float4), hipMemcpyHostToDevice), "mesh upload") ||
        !hip_ok(hipMemcpy((float4*)tp32.p + 4 * tri_used, pk32.data(), 4 * npad * sizeof(float4), hipMemcpyHostToDevice), "mesh upload") ||
        !hip_ok(hipMemcpy((double2*)tp64.p + 5 * tri_used, pk64.data(), 5 * npad * sizeof(double2), hipMemcpyHostToDevice), "mesh upload") ||
        !hip_ok(hipMemcpy((float4*)tsp.p + tile_used, tsph.data(), ntile * sizeof(float4), hipMemcpyHostToDevice), "mesh upload"))
        return MCD_E_HIP;
    tri_used += npad;
    tile_used += ntile;
    mi.alive = true;
    int32_t mid = (int32_t)meshes.size();
    meshes.push_back(mi);
    mcd_status st = upload_meshes();
    if (st != MCD_OK) return st;
    *id = mid;
    return MCD_OK;
}

TriStore Ctx::store() const
{
    TriStore S;
    S.v32 = (float*)t32.p;
    S.v64 = (double*)t64.p;
    S.orig = (int32_t*)torig.p;
    S.pos = (int32_t*)tpos.p;
    S.tile_sph = (float4*)tsp.p;
    S.grp_sph = (float4*)gsp.p;
    S.tri_sph = (float4*)trs.p;
    S.p32 = (float4*)tp32.p;
    S.p64 = (double2*)tp64.p;
    S.cap = tri_cap;
    return S;
}

mcd_status Ctx::particles_set(int32_t n, const int32_t* pid, const int32_t* mesh_id, const mcd_state* s)
{
    if (n < 0 || (n > 0 && (!pid || !mesh_id || !s))) { err = "particles_set: invalid arguments"; return MCD_E_INVALID; }
    for (int i = 0; i < n; ++i) {
        if (pid[i] < 0) { err = "particles_set: negative particle id"; return MCD_E_INVALID; }
        if (mesh_id[i] < 0 || mesh_id[i] >= (int32_t)meshes.size() || !meshes[mesh_id[i]].alive) {
            err = "particles_set: unknown mesh id " + std::to_string(mesh_id[i]);
            return MCD_E_NOT_FOUND;
        }
        const double* d = &s[i].x[0];
        for (int k = 0; k < 13; ++k)
            if (!std::isfinite(d[k])) { err = "particles_set: non-finite state"; return MCD_E_INVALID; }
        double qn = std::sqrt(s[i].q[0] * s[i].q[0] + s[i].q[1] * s[i].q[1] + s[i].q[2] * s[i].q[2] + s[i].q[3] * s[i].q[3]);
        if (!(qn > 0)) { err = "particles_set: zero quaternion"; return MCD_E_INVALID; }
    }
    wait_no_readers();
    for (int i = 0; i < n; ++i) {
        Particle p;
        p.mesh = mesh_id[i];
        p.s = s[i];
        double qn = std::sqrt(p.s.q[0] * p.s.q[0] + p.s.q[1] * p.s.q[1] + p.s.q[2] * p.s.q[2] + p.s.q[3] * p.s.q[3]);
        for (int k = 0; k < 4; ++k) p.s.q[k] /= qn;
        particles[pid[i]] = p;
    }
    return upload_particles(n, pid);
}


// ---------------------------------------------------------------- queries
// Source record of a pair: the state snapshots and mesh records, copied
// (the FP64 preparation runs on the device, k_pair_prep).
static void make_src(PairSrc& Q, const MeshInfo& ma, const MeshInfo& mb, const mcd_state& sa,
                     const mcd_state& sb, double t)
{
    std::memset(&Q, 0, sizeof Q);
    std::memcpy(Q.sa, &sa.x[0], sizeof Q.sa);
    std::memcpy(Q.sb, &sb.x[0], sizeof Q.sb);
    Q.t = t;
    Q.halo_a = ma.halo; Q.halo_b = mb.halo;
    Q.rad_a = ma.radius; Q.rad_b = mb.radius;
    Q.emax_a = ma.emax; Q.emax_b = mb.emax;
    Q.tri0_a = (int32_t)ma.tri0; Q.tri0_b = (int32_t)mb.tri0;
    Q.na = ma.nt; Q.nb = mb.nt;
    Q.tile0_a = (int32_t)ma.tile0; Q.tile0_b = (int32_t)mb.tile0;
    Q.nta = ma.ntile; Q.ntb = mb.ntile;
    Q.group0_a = (int32_t)ma.group0; Q.group0_b = (int32_t)mb.group0;
}

static uint64_t dbits(double v)
{
    uint64_t u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}

PrepOpts Ctx::prep_opts(const mcd_qopts& o) const
{
    PrepOpts p{};
    p.dt = o.dt;
    p.tol_rel = o.tol_rel;
    p.margin_c = margin_c;
    p.samples = o.samples;
    p.flags = (int32_t)o.flags;
    return p;
}

// Pinned staging of a query's pair sources (header with the pair count, then
// the records) with each pair's offset tp0: the first word of its tile-cull
// bitmask (contact sets) or its first entry in the tile-pair list (time
// stamps). total = bitmask words or tile pairs of the query.
mcd_status Ctx::stage_src(const Query& q, Slot& s, int32_t cap, bool toi, int64_t& total)
{
    const int32_t n = (int32_t)q.src.size();
    mcd_status st;
    if ((st = s.ws.src.reserve(PAIR_HDR + sizeof(PairSrc) * (size_t)std::max(cap, 1), s.err)) != MCD_OK ||
        (st = s.ws.h_src.reserve(PAIR_HDR + sizeof(PairSrc) * (size_t)std::max(cap, 1), s.err)) != MCD_OK)
        return st;
    std::memset(s.ws.h_src.p, 0, PAIR_HDR);
    ((int32_t*)s.ws.h_src.p)[0] = n;
    PairSrc* hs = (PairSrc*)((char*)s.ws.h_src.p + PAIR_HDR);
    if (n > 0) std::memcpy(hs, q.src.data(), sizeof(PairSrc) * n);
    total = 0;
    for (int i = 0; i < n; ++i) {
        hs[i].tp0 = total;
        const int64_t tp = (int64_t)hs[i].nta * hs[i].ntb;
        total += toi ? tp : (tp + 63) / 64;
    }
    return MCD_OK;
}

mcd_status Ctx::check_opts(const mcd_qopts* o, mcd_qopts& q)
{
    q = o ? *o : mcd_qopts{};
    if (q.flags == 0) q.flags = MCD_Q_MIXED;
    const uint32_t known = MCD_Q_FP64 | MCD_Q_MIXED | MCD_Q_DENSE | MCD_Q_TIMING | MCD_Q_CLOSEST |
                           MCD_Q_CONTACTS | MCD_Q_VALIDATE | MCD_Q_NARROW | MCD_Q_FUSE | MCD_Q_DEVICE_OUT;
    if ((q.flags & (MCD_Q_FP64 | MCD_Q_MIXED)) == (MCD_Q_FP64 | MCD_Q_MIXED) || (q.flags & ~known) != 0) {
        err = "query: unknown flags, or FP64 and MIXED together";
        return MCD_E_INVALID;
    }
    if (!(q.flags & (MCD_Q_FP64 | MCD_Q_MIXED))) q.flags |= MCD_Q_MIXED;
    if (!(q.flags & (MCD_Q_CLOSEST | MCD_Q_CONTACTS))) q.flags |= MCD_Q_CLOSEST | MCD_Q_CONTACTS;
    if ((q.flags & MCD_Q_VALIDATE) && ((q.flags & (MCD_Q_FP64 | MCD_Q_DENSE)) || q.dt != 0.0)) {
        err = "query: MCD_Q_VALIDATE applies to static MIXED contact-set queries only";
        return MCD_E_INVALID;
    }
    if (!(q.dt >= 0.0) || !std::isfinite(q.dt)) { err = "query: dt must be finite and >= 0"; return MCD_E_INVALID; }
    if ((q.flags & MCD_Q_NARROW) && (q.dt == 0.0 || (q.flags & MCD_Q_DENSE))) {
        err = "query: MCD_Q_NARROW applies to time queries (dt > 0) without MCD_Q_DENSE";
        return MCD_E_INVALID;
    }
    if ((q.flags & MCD_Q_DEVICE_OUT) &&
        (q.dt != 0.0 || (q.flags & (MCD_Q_CLOSEST | MCD_Q_CONTACTS)) != (MCD_Q_CLOSEST | MCD_Q_CONTACTS))) {
        err = "query: MCD_Q_DEVICE_OUT applies to static queries that return both closest points and contacts";
        return MCD_E_INVALID;
    }
    if (q.samples == 0) q.samples = 64;
    if (q.tol_rel == 0.0) q.tol_rel = 1e-6;
    if (q.samples < 1 || q.samples > 128 || !(q.tol_rel >= 1e-7 && q.tol_rel < 1.0)) {
        err = "query: samples must be in [1, 128] and tol_rel in [1e-7, 1)";
        return MCD_E_INVALID;
    }
    return MCD_OK;
}

// Snapshot the pairs' meshes and states and compute their parameters.
// Host threads for splitting large copies and preparations: the machine's
// count, read once (each query would otherwise read it from the system).
static unsigned host_threads()
{
    static const unsigned n = std::max(1u, std::thread::hardware_concurrency());
    return n;
}

mcd_status Ctx::prepare_pairs(const int32_t* pp, int32_t n, Query& q, std::string& err)
{
    const mcd_qopts& o = q.opts;
    q.pairs.assign(pp, pp + 2 * (size_t)n);
    q.src.resize(n);
    q.mi.resize(2 * (size_t)n);
    q.st.resize(2 * (size_t)n);
    q.tile_pairs_total = 0;
    q.tri_pairs_covered = 0;
    // Pairs [lo, hi): snapshots and pair sources. The particle and mesh
    // tables are only read here (the API lock is held), so large lists are
    // split over a few host threads; each part stops at its first bad pair
    // and the lowest such pair is reported.
    struct Part {
        int64_t tiles = 0, tris = 0;
        int bad = INT32_MAX;
        mcd_status st = MCD_OK;
        std::string err;
    };
    auto run = [&](int lo, int hi, Part& r) {
        for (int i = lo; i < hi; ++i) {
            auto ia = particles.find(pp[2 * i]), ib = particles.find(pp[2 * i + 1]);
            if (ia == particles.end() || ib == particles.end()) {
                r = Part{0, 0, i, MCD_E_NOT_FOUND, "query: unknown particle id in pair " + std::to_string(i)};
                return;
            }
            if (pp[2 * i] == pp[2 * i + 1]) {
                r = Part{0, 0, i, MCD_E_INVALID, "query: pair " + std::to_string(i) + " repeats a particle"};
                return;
            }
            const Particle &A = ia->second, &B = ib->second;
            const MeshInfo &ma = meshes[A.mesh], &mb = meshes[B.mesh];
            if (!ma.alive || !mb.alive) {
                r = Part{0, 0, i, MCD_E_NOT_FOUND, "query: pair " + std::to_string(i) + " uses an unloaded mesh"};
                return;
            }
            q.mi[2 * i] = ma; q.mi[2 * i + 1] = mb;
            q.st[2 * i] = A.s; q.st[2 * i + 1] = B.s;
            make_src(q.src[i], ma, mb, A.s, B.s, 0.0);
            if (o.dt > 0.0) q.src[i].table0 = (int64_t)i * (o.samples + 1);
            r.tiles += (int64_t)ma.ntile * mb.ntile;
            r.tris += (int64_t)ma.nt * mb.nt;
        }
    };
    const int nt = n < 4096 ? 1 : (int)std::min<int64_t>({8, (int64_t)host_threads(), (int64_t)n / 2048});
    Part parts[8];
    if (nt <= 1) {
        run(0, n, parts[0]);
    } else {
        // parts whose thread cannot be started run here
        std::vector<std::thread> ts;
        ts.reserve(nt - 1);
        int started = 1;
        try {
            for (; started < nt; ++started)
                ts.emplace_back(run, (int)((int64_t)n * started / nt), (int)((int64_t)n * (started + 1) / nt),
                                std::ref(parts[started]));
        } catch (const std::system_error&) {
        }
        for (int t = started; t < nt; ++t) run((int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt), parts[t]);
        run(0, (int)((int64_t)n / nt), parts[0]);
        for (auto& t : ts) t.join();
    }
    for (int t = 0; t < nt; ++t) {   // in pair order: the first bad part holds the lowest bad pair
        const Part& r = parts[t];
        if (r.st != MCD_OK) { err = r.err; return r.st; }
        q.tile_pairs_total += r.tiles;
        q.tri_pairs_covered += r.tris;
    }
    // Device working set of the query (items, partials and per-pair arrays).
    q.mem_estimate = q.tile_pairs_total * 48 +
                     (int64_t)n * (1024 + (o.dt > 0.0 ? (int64_t)(o.samples + 1) * 144 : 0));
    return MCD_OK;
}

// Candidate pairs inside a cluster (section 2, clustering): bounding spheres
// about the rotation centres (radius = largest vertex distance, unchanged by
// rotation) closer than R_a + R_b + eps_a + eps_b, at the start (static) or
// at the closest approach of the linear centre paths over [0, dt]. A uniform
// hash grid finds neighbours; pairs are listed in cluster order (a < b).
mcd_status Ctx::cluster_pairs(int32_t n, const int32_t* pid, const mcd_state* states,
                              const mcd_qopts& o, std::vector<int32_t>& out)
{
    if (n < 0 || (n > 0 && !pid)) { err = "query_cluster: invalid arguments"; return MCD_E_INVALID; }
    if (states) {
        std::vector<int32_t> mids(n);
        for (int i = 0; i < n; ++i) {
            auto it = particles.find(pid[i]);
            if (it == particles.end()) { err = "query_cluster: unknown particle " + std::to_string(pid[i]); return MCD_E_NOT_FOUND; }
            mids[i] = it->second.mesh;
        }
        mcd_status st = particles_set(n, pid, mids.data(), states);
        if (st != MCD_OK) return st;
    }
    std::vector<const Particle*> P(n);
    double reach = 0, vmax = 0, hmax = 0;
    for (int i = 0; i < n; ++i) {
        auto it = particles.find(pid[i]);
        if (it == particles.end()) { err = "query_cluster: unknown particle " + std::to_string(pid[i]); return MCD_E_NOT_FOUND; }
        P[i] = &it->second;
        const MeshInfo& m = meshes[P[i]->mesh];
        reach = std::max(reach, m.radius);
        hmax = std::max(hmax, m.halo);
        const double* v = P[i]->s.v;
        vmax = std::max(vmax, std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    }
    {
        std::vector<int32_t> ids(pid, pid + n);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end()) {
            err = "query_cluster: particle listed twice";
            return MCD_E_INVALID;
        }
    }
    const double cell = 2.0 * reach + 2.0 * hmax + 2.0 * vmax * o.dt + 1e-9;
    // uniform grid as sorted (cell key, particle) pairs; a particle's
    // neighbours are found in the 27 cells around it by binary search
    auto key = [&](int64_t a, int64_t b, int64_t c) { return ((a & 0x1fffff) << 42) | ((b & 0x1fffff) << 21) | (c & 0x1fffff); };
    std::vector<int64_t> ci(3 * (size_t)n);
    std::vector<std::pair<int64_t, int32_t>> cells(n);
    for (int i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) ci[3 * i + c] = (int64_t)std::floor(P[i]->s.x[c] / cell);
        cells[i] = {key(ci[3 * i], ci[3 * i + 1], ci[3 * i + 2]), i};
    }
    std::sort(cells.begin(), cells.end());
    std::vector<std::pair<int32_t, int32_t>> found;
    for (int i = 0; i < n; ++i)
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    const int64_t k = key(ci[3 * i] + dx, ci[3 * i + 1] + dy, ci[3 * i + 2] + dz);
                    auto g = std::lower_bound(cells.begin(), cells.end(), std::make_pair(k, (int32_t)-1));
                    for (; g != cells.end() && g->first == k; ++g) {
                        const int j = g->second;
                        if (j <= i) continue;
                        const Particle &A = *P[i], &B = *P[j];
                        const MeshInfo &ma = meshes[A.mesh], &mb = meshes[B.mesh];
                        const double lim = ma.radius + mb.radius + ma.halo + mb.halo;
                        double d[3], dv[3], vv = 0, dvx = 0;
                        for (int c = 0; c < 3; ++c) {
                            d[c] = B.s.x[c] - A.s.x[c];
                            dv[c] = B.s.v[c] - A.s.v[c];
                            vv += dv[c] * dv[c];
                            dvx += d[c] * dv[c];
                        }
                        double t = 0.0;
                        if (o.dt > 0.0 && vv > 0.0) t = std::min(o.dt, std::max(0.0, -dvx / vv));
                        double r2 = 0;
                        for (int c = 0; c < 3; ++c) r2 += (d[c] + dv[c] * t) * (d[c] + dv[c] * t);
                        if (r2 <= lim * lim) found.push_back({i, j});
                    }
                }
    std::sort(found.begin(), found.end());
    out.clear();
    out.reserve(2 * found.size());
    for (auto& f : found) { out.push_back(pid[f.first]); out.push_back(pid[f.second]); }
    return MCD_OK;
}

mcd_status Ctx::enqueue(std::shared_ptr<Query> q, uint64_t* ticket)
{
    if (q->mem_estimate > mem_budget) {
        err = "query: needs about " + std::to_string(q->mem_estimate) +
              " bytes of working memory, more than the budget of " + std::to_string(mem_budget);
        return MCD_E_BUSY;
    }
    const uint64_t t = next_ticket++;
    tickets[t] = q;
    q->t_submit = std::chrono::steady_clock::now();
    if (q->dev && q->npairs() > 0) {
        std::lock_guard<std::mutex> lk(rd_mtx);
        ++dev_readers;
    }
    if (q->npairs() == 0) {
        std::lock_guard<std::mutex> lk(q->m);
        q->stats.graph_captures = graph_captures.load();
        q->done = true;
    } else {
        std::lock_guard<std::mutex> lk(qmtx);
        pending.push_back(q);
    }
    qcv.notify_all();
    *ticket = t;
    return MCD_OK;
}

std::shared_ptr<Query> Ctx::find(uint64_t t)
{
    auto it = tickets.find(t);
    if (it == tickets.end()) { err = "unknown ticket " + std::to_string(t); return nullptr; }
    return it->second;
}

// ---------------------------------------------------------------- execution
// Queries batch together when they have the same options and kind: host
// pair lists with host pair lists, device cluster queries (static) with
// device cluster queries; a device pair list runs alone.
static bool same_kind(const Query& qa, const Query& qb)
{
    const mcd_qopts &a = qa.opts, &b = qb.opts;
    if ((a.flags | b.flags) & MCD_Q_DEVICE_OUT) return false;   // results held per query on the device
    const bool kinds = (!qa.dev && !qb.dev) || (qa.cluster && qb.cluster && a.dt == 0.0);
    return kinds && a.dt == b.dt && a.flags == b.flags && a.samples == b.samples && a.tol_rel == b.tol_rel;
}

void Ctx::worker(int i)
{
    Slot& s = *slots[i];
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<std::shared_ptr<Query>> batch;
        int64_t mem = 0;
        {
            std::unique_lock<std::mutex> lk(qmtx);
            qcv.wait(lk, [&] {
                return (stopping && pending.empty()) ||
                       (!pending.empty() &&
                        (mem_inflight == 0 || mem_inflight + pending.front()->mem_estimate <= mem_budget));
            });
            if (pending.empty()) return;
            auto q0 = pending.front();
            pending.pop_front();
            batch.push_back(q0);
            mem = q0->mem_estimate;
            int64_t np = (int64_t)q0->npairs();
            while (!pending.empty()) {
                auto& q = pending.front();
                if (!same_kind(*q, *q0) || np + (int64_t)q->npairs() > max_batch_pairs ||
                    mem_inflight + mem + q->mem_estimate > mem_budget)
                    break;
                mem += q->mem_estimate;
                np += (int64_t)q->npairs();
                batch.push_back(q);
                pending.pop_front();
            }
            mem_inflight += mem;
        }
        {
            std::shared_lock<std::shared_mutex> slk(store_mtx);
            run_batch(batch, s);
        }
        {
            std::lock_guard<std::mutex> lk(qmtx);
            mem_inflight -= mem;
        }
        qcv.notify_all();
    }
}

static void finish(Query& q, mcd_status st, const std::string& err, int32_t nq, int32_t np, int64_t captures)
{
    q.stats.graph_captures = captures;
    q.stats.latency_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                   q.t_submit).count();
    q.stats.batch_queries = nq;
    q.stats.batch_pairs = np;
    std::lock_guard<std::mutex> lk(q.m);
    q.status = st;
    if (st != MCD_OK) q.err = err;
    q.done = true;
    q.cv.notify_all();
}

// Run the queries of a batch as one pair list and split the results. Every
// pair is computed independently of the others, so a query's results are the
// same alone and in any batch.
// The contact records of batch pairs [lo, hi) for query q: a range of the
// batch's pinned buffer, shared (no copy); records held elsewhere are copied
// and re-based.
static void slice_contacts(Query& all, const std::shared_ptr<HostBuf>& share, int32_t lo, int32_t hi, Query& q)
{
    mcd_contact* cb = all.cdata();
    mcd_contact* ce = cb + all.ncon;
    auto c0 = std::lower_bound(cb, ce, lo, [](const mcd_contact& c, int32_t v) { return c.pair < v; });
    auto c1 = std::lower_bound(c0, ce, hi, [](const mcd_contact& c, int32_t v) { return c.pair < v; });
    q.ncon = (int64_t)(c1 - c0);
    if (share) {
        q.cshare = share;
        q.coff = (int64_t)(c0 - cb);
        q.pair_base = lo;
        q.rebased = lo == 0;
    } else {
        q.cvec.assign(c0, c1);
        for (auto& c : q.cvec) c.pair -= lo;
    }
}

// The batch's pinned contact buffer as a shared lease that returns it to the
// pool when the last query holding it is released.
static std::shared_ptr<HostBuf> share_contacts(Query& all, PinnedPool* pool)
{
    if (!all.cpin || all.ncon == 0) return nullptr;
    HostBuf* hb = all.cpin;
    all.cpin = nullptr;
    std::shared_ptr<HostBuf> sp(hb, [pool](HostBuf* b) { pool->put(b); });
    all.cshare = sp;
    all.coff = 0;
    return sp;
}

void Ctx::run_batch(std::vector<std::shared_ptr<Query>>& batch, Slot& s)
{
    const bool toi = batch[0]->opts.dt > 0.0;
    if (batch.size() == 1) {
        Query& q = *batch[0];
        mcd_status st = toi ? run_toi(q, s) : run_static(q, s);
        const bool dev = q.dev;
        finish(q, st, s.err, 1, q.cluster ? (int32_t)(q.pairs.size() / 2) : q.npairs(), graph_captures.load());
        if (dev) reader_done();
        return;
    }
    if (batch[0]->cluster) {
        run_cluster_batch(batch, s);
        return;
    }
    Query all;
    all.pool = &pinned;
    all.opts = batch[0]->opts;
    std::vector<int32_t> off;
    for (auto& qp : batch) {
        Query& q = *qp;
        off.push_back((int32_t)all.src.size());
        for (size_t i = 0; i < q.src.size(); ++i) {
            PairSrc P = q.src[i];
            if (toi) P.table0 = (int64_t)all.src.size() * (all.opts.samples + 1);
            all.src.push_back(P);
        }
        all.pairs.insert(all.pairs.end(), q.pairs.begin(), q.pairs.end());
        all.mi.insert(all.mi.end(), q.mi.begin(), q.mi.end());
        all.st.insert(all.st.end(), q.st.begin(), q.st.end());
        all.tile_pairs_total += q.tile_pairs_total;
        all.tri_pairs_covered += q.tri_pairs_covered;
    }
    off.push_back((int32_t)all.src.size());
    mcd_status st = toi ? run_toi(all, s) : run_static(all, s);
    const std::shared_ptr<HostBuf> share = st == MCD_OK ? share_contacts(all, &pinned) : nullptr;
    for (size_t b = 0; b < batch.size(); ++b) {
        Query& q = *batch[b];
        if (st == MCD_OK) {
            const int32_t lo = off[b], hi = off[b + 1];
            q.result.assign(all.result.begin() + lo, all.result.begin() + hi);
            slice_contacts(all, share, lo, hi, q);
            const double sub = q.stats.submit_ms;
            q.stats = all.stats;
            q.stats.submit_ms = sub;
        }
        finish(q, st, s.err, (int32_t)batch.size(), (int32_t)all.src.size(), graph_captures.load());
    }
}

// Device cluster queries of a batch: their member lists become segments of
// one list, the broad phase pairs members inside a segment only, and the
// results are split by each segment's pair range.
void Ctx::run_cluster_batch(std::vector<std::shared_ptr<Query>>& batch, Slot& s)
{
    Query all;
    all.pool = &pinned;
    all.opts = batch[0]->opts;
    all.dev = all.cluster = true;
    all.seg_off.push_back(0);
    int64_t cap = 0;
    for (auto& qp : batch) {
        all.members.insert(all.members.end(), qp->members.begin(), qp->members.end());
        all.seg_off.push_back((int32_t)all.members.size());
        cap += qp->n_dev;
        all.tile_pairs_total += qp->tile_pairs_total;
    }
    all.n_dev = (int32_t)std::min<int64_t>(cap, INT32_MAX);
    mcd_status st = run_static(all, s);
    const int32_t np_all = (int32_t)(all.pairs.size() / 2);
    const std::shared_ptr<HostBuf> share = st == MCD_OK ? share_contacts(all, &pinned) : nullptr;
    for (size_t b = 0; b < batch.size(); ++b) {
        Query& q = *batch[b];
        if (st == MCD_OK) {
            const int32_t lo = np_all ? (int32_t)all.seg_pairs[b] : 0, hi = np_all ? (int32_t)all.seg_pairs[b + 1] : 0;
            q.pairs.assign(all.pairs.begin() + 2 * (size_t)lo, all.pairs.begin() + 2 * (size_t)hi);
            q.result.assign(all.result.begin() + lo, all.result.begin() + hi);
            slice_contacts(all, share, lo, hi, q);
            const double sub = q.stats.submit_ms;
            q.stats = all.stats;
            q.stats.submit_ms = sub;
        }
        finish(q, st, s.err, (int32_t)batch.size(), np_all, graph_captures.load());
        reader_done();
    }
}

// Launch shapes the autotuner chooses from: waves per CU of the near-list
// stage and of the evaluation stage (both persistent: a grid larger than the
// chip holds waits for free slots; a smaller one leaves CUs idle on large
// queries but launches and drains faster on small ones).
static const Shape kShapes[] = {{32, 24}, {16, 16}, {32, 16}, {16, 24}, {8, 8}, {4, 4}};
static constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
static constexpr int kTuneReps = 2;

// Bucket of a static query for the autotuner: precision and the binary
// order of magnitude of its tile pairs.
static uint32_t tune_bucket(bool fp64, int64_t tile_pairs)
{
    uint32_t lg = 0;
    while (lg < 40 && ((int64_t)1 << (lg + 1)) <= tile_pairs) ++lg;
    return (fp64 ? 0x100u : 0u) | lg;
}

int Ctx::pick_shape(uint32_t bucket, bool& measure)
{
    measure = false;
    if (!use_tune) return 0;
    std::lock_guard<std::mutex> lk(tune_mtx);
    TuneEntry& t = tune[bucket];
    if (t.ms.empty()) t.ms.assign(kNumShapes, INFINITY);
    if (t.best >= 0) return t.best;
    // candidates in turn, each measured kTuneReps times (minimum kept)
    const int c = t.next % kNumShapes;
    ++t.next;
    measure = true;
    return c;
}

void Ctx::report_shape(uint32_t bucket, int shape, float ms)
{
    std::lock_guard<std::mutex> lk(tune_mtx);
    TuneEntry& t = tune[bucket];
    if (t.best >= 0) return;
    t.ms[shape] = std::min(t.ms[shape], ms);
    if (++t.reports >= kNumShapes * kTuneReps) {
        int b = 0;
        for (int i = 1; i < kNumShapes; ++i)
            if (t.ms[i] < t.ms[b]) b = i;
        t.best = b;
    }
}

int Ctx::tune_pending(uint32_t bucket)
{
    if (!use_tune) return 0;
    std::lock_guard<std::mutex> lk(tune_mtx);
    auto it = tune.find(bucket);
    if (it == tune.end()) return kNumShapes * kTuneReps;
    if (it->second.best >= 0) return 0;
    return std::max(0, kNumShapes * kTuneReps - it->second.reports);
}

mcd_status Ctx::run_static(Query& q, Slot& s)
{
    // A device pair list (q.dev) is gathered into pair sources on the device,
    // in the captured chain; its tile-pair total is known after a run, and a
    // run whose totals exceed the buffers is repeated with larger ones.
    // A device cluster query (q.cluster) finds its pairs on the device first;
    // until that run has counted them, n is the capacity of the pair list.
    const bool dev = q.dev, cluster = q.cluster;
    int32_t n = q.npairs();
    q.stats.tile_pairs_total = q.tile_pairs_total;
    q.stats.tri_pairs_covered = q.tri_pairs_covered;
    if (n == 0) {
        q.result.clear();
        q.ncon = 0;
        return MCD_OK;
    }
    const bool fp64 = (q.opts.flags & MCD_Q_FP64) != 0;
    const bool dense = (q.opts.flags & MCD_Q_DENSE) != 0;
    // device lists are bucketed apart, on their estimate of 64 tile pairs
    // per pair (their count is known only after the run)
    // (and the second phases of time-stamp queries, whose estimate counts
    // the tile pairs of every pair)
    const int64_t grid_tp = q.grid_tile_pairs >= 0 ? q.grid_tile_pairs : q.tile_pairs_total;
    const uint32_t bucket = tune_bucket(fp64, grid_tp) | (dev ? 0x200u : 0u) | (q.staged ? 0x400u : 0u);
    bool measure = false;
    const int shape = dense ? 0 : pick_shape(bucket, measure);
    const bool timing = measure || (q.opts.flags & MCD_Q_TIMING) != 0;
    Launch L{s.stream, num_cu};
    std::string& e = s.err;
    mcd_status st;
    if (dev && !cluster) {
        // the caller's list becomes readable when its stream reaches the event
        if (!s.hip_ok(hipStreamWaitEvent(s.stream, q.ready, 0), "wait for the pair list")) return MCD_E_HIP;
        q.pairs.resize(2 * (size_t)n);
    }
    // counters: 0 items, 1 candidates, 2 refine items, 3 re-decided records,
    // 4/5 work queues, 6 records of the near list (plane survivors), 8-9
    // tiled triangle pairs, 10-11 evaluations, 12-13 dense FP64 evaluations,
    // 14-15 sphere tests, 16-17 contacts, 18-19 near pairs, 20 the largest
    // contact segment, 21 pairs with more than 64 contacts, 22-23 offset units
    // of a device list, 24-25 guard-band pairs, 26-27 validated pairs, 29
    // device-list errors, 30-31 tile pairs and 32-33 triangle pairs of a device
    // list, 34-35 the largest margin ratios, 36-37 the pairs of a device
    // broad phase, 38-39 sphere tests of the tile cull, 64-191 the near
    // stage's per-XCD queues
    for (int attempt = 0; attempt < 8; ++attempt) {
        // persistent grids, capped for small queries at about one wave per
        // 16 tile pairs of the query (an upper bound of its kept items): a
        // wave without work still costs its launch and queue probes. The cap
        // is a power of two, so queries of similar size share one captured
        // chain instead of each capturing its own.
        int64_t gcap = 4;
        while (gcap < (grid_tp + 31) / 32) gcap <<= 1;
        const int gnear = (int)std::min<int64_t>(num_cu * kShapes[shape].near_wpc, gcap);
        const int geval = (int)std::min<int64_t>(num_cu * kShapes[shape].eval_wpc, 2 * gcap);
        if (q.tile_pairs_total > s.item_cap)
            s.item_cap = std::max<int64_t>(q.tile_pairs_total, s.item_cap + s.item_cap / 2);
        const int64_t item_cap = std::max<int64_t>(1, s.item_cap);
        if (cluster) n = q.n_dev;
        if (n > s.pair_cap) s.pair_cap = std::max(n, s.pair_cap + s.pair_cap / 2);
        const int32_t pc = s.pair_cap;
        const int64_t cc = s.cand_cap, oc = s.cand_cap, nc = dense ? 1 : s.near_cap;
        if ((st = s.ws.pairs.reserve(PAIR_HDR + sizeof(PairDev) * pc, e)) != MCD_OK ||
            (st = s.ws.items.reserve((dense ? sizeof(Item) : sizeof(NearItem)) * item_cap, e)) != MCD_OK ||
            (st = s.ws.refs.reserve(sizeof(Item) * (dense ? item_cap : 1), e)) != MCD_OK ||
            (st = s.ws.part32.reserve(sizeof(PartialF) * (dense ? item_cap : 1), e)) != MCD_OK ||
            (st = s.ws.part64.reserve(sizeof(PartialD) * (dense ? item_cap : 1), e)) != MCD_OK ||
            (st = s.ws.near.reserve(sizeof(NearRec) * nc, e)) != MCD_OK ||
            (st = s.ws.cands.reserve(sizeof(Cand) * cc, e)) != MCD_OK ||
            (st = s.ws.outs.reserve(sizeof(CandOut) * oc, e)) != MCD_OK ||
            (st = s.ws.pair_ub.reserve(sizeof(uint32_t) * pc, e)) != MCD_OK ||
            (st = s.ws.pair_d2.reserve(sizeof(uint64_t) * pc, e)) != MCD_OK ||
            (st = s.ws.pair_tie.reserve(sizeof(uint64_t) * pc, e)) != MCD_OK ||
            (st = s.ws.pair_cnt.reserve(sizeof(int32_t) * pc, e)) != MCD_OK ||
            (st = s.ws.pair_off.reserve(sizeof(int32_t) * ((size_t)pc + 1), e)) != MCD_OK ||
            (st = s.ws.large.reserve(sizeof(int32_t) * (size_t)pc, e)) != MCD_OK ||
            (st = s.ws.seg.reserve(sizeof(uint64_t) * cc, e)) != MCD_OK ||
            (st = s.ws.ckey.reserve(sizeof(uint64_t) * cc, e)) != MCD_OK ||
            (st = s.ws.cd2.reserve(sizeof(uint64_t) * cc, e)) != MCD_OK ||
            (st = s.ws.cullmask.reserve(sizeof(uint64_t) * ((size_t)item_cap / 64 + pc + 1), e)) != MCD_OK ||
            (st = s.ws.pair_out.reserve(sizeof(PairOut) * pc, e)) != MCD_OK ||
            (st = s.ws.counters.reserve(sizeof(int32_t) * NCOUNTERS, e)) != MCD_OK ||
            (st = s.ws.stats.reserve(sizeof(uint64_t) * STAT_ROWS * STAT_WAVES, e)) != MCD_OK ||
            (st = s.ws.scan.reserve(cull_scan_bytes(pc), e)) != MCD_OK ||
            (st = s.ws.h_counters.reserve(sizeof(int32_t) * 64, e)) != MCD_OK ||
            (st = s.ws.h_pair_out.reserve(sizeof(PairOut) * pc, e)) != MCD_OK)
            return st;
        // pair sources with each pair's first word of the tile-cull bitmask:
        // staged by the host, or gathered on the device from the device list
        const int64_t word_cap = item_cap / 64 + pc + 1;
        if (q.staged) {
            // the first phase's sources, on the device already
        } else if (!dev) {
            int64_t nwords = 0;
            if ((st = stage_src(q, s, pc, false, nwords)) != MCD_OK) return st;
            if (nwords > word_cap) { e = "query: tile-cull bitmask overflow"; return MCD_E_INVALID; }
        } else {
            if ((st = s.ws.src.reserve(PAIR_HDR + sizeof(PairSrc) * (size_t)pc, e)) != MCD_OK ||
                (st = s.ws.h_src.reserve(PAIR_HDR, e)) != MCD_OK ||
                (st = s.ws.dlist.reserve(PAIR_HDR + sizeof(int32_t) * 2 * (size_t)pc, e)) != MCD_OK ||
                (st = s.ws.gather_tmp.reserve(sizeof(int64_t) * 2 * (size_t)pc, e)) != MCD_OK)
                return st;
            std::memset(s.ws.h_src.p, 0, PAIR_HDR);
            ((int32_t*)s.ws.h_src.p)[0] = n;
            if (cluster && (st = stage_members(s.ws.bp, s.stream, q.members, q.seg_off, pc, e)) != MCD_OK) return st;
        }
        const int32_t* nlist = (const int32_t*)s.ws.dlist.p;
        const int32_t* dlist = (const int32_t*)((const char*)s.ws.dlist.p + PAIR_HDR);
        BpBufs& bp = s.ws.bp;
        const int32_t mcap = cluster ? (int32_t)(bp.mem.bytes / sizeof(BpMember)) : 0;
        const int32_t seg_cap = cluster ? (int32_t)(bp.seg.bytes / sizeof(int32_t)) - 1 : 0;
        const PrepOpts popt = prep_opts(q.opts);
        const int32_t* nq = (const int32_t*)s.ws.pairs.p;
        PairDev* dp = pairs_dev(s.ws);
        int32_t* c = (int32_t*)s.ws.counters.p;
        unsigned long long* c64 = (unsigned long long*)c;
        TriStore S = store();
        hipEvent_t* ev = s.ev;
        NearRec* nr = (NearRec*)s.ws.near.p;
        unsigned long long* sl = (unsigned long long*)s.ws.stats.p;
        // per-wave counts: row 0 sphere tests (k_near, two blocks per grid
        // unit), row 1 evaluations of the main pass, row 2 the FP64 refine
        // pass, row 3 the contacts of the FP64 re-decision, row 4 the near
        // pairs (plane-separation tests of k_near)
        const int grec = recheck_grid(cc);
        StatPlan plan{};
        // row 5 the re-decided pairs in the guard band, row 6 the FP32
        // estimates compared by a validating query
        // and row 7 the sphere tests of the tile cull (both levels)
        if (!dense) plan = StatPlan{8, {2 * gnear, geval, 0, grec, 2 * gnear, grec, grec, cull_grid(L, pc)},
                                    {7, 5, 6, 8, 9, 12, 13, 19}};
        else if (!fp64) plan = StatPlan{7, {0, grid32, grid64, grec, 0, grec, grec}, {7, 5, 6, 8, 9, 12, 13}};
        else plan = StatPlan{7, {0, grid64, 0, grec, 0, grec, grec}, {7, 5, 6, 8, 9, 12, 13}};
        for (int i = 0; i < plan.n; ++i)
            if (plan.waves[i] > STAT_WAVES) { e = "query: grid exceeds the counter slots"; return MCD_E_INVALID; }
        Item* ties = fp64 ? (Item*)s.ws.items.p : (Item*)s.ws.refs.p;
        int32_t* tie_count = fp64 ? c + 0 : c + 2;
        // The kernel chain from the reset of the counters to the per-pair
        // results. Contact-set queries: tile cull, near list, one evaluation
        // per near pair (FP32 filter or exact FP64). Dense queries evaluate
        // every triangle pair of every tile pair and keep per-item minima;
        // mixed dense queries re-run in FP64 the items that can hold a pair's
        // minimum. The FP64 re-decision of the candidates yields the
        // contacts, and a pair in contact has its minimum among them; ties in
        // the minimum are settled once every minimum is final. With events,
        // ev 5 / 6 / 2 / 3 bracket the stages for per-kernel times.
        auto chain = [&](bool events) -> bool {
            auto mark = [&](int i) { return !events || s.hip_ok(hipEventRecord(ev[i], s.stream), "event"); };
            bool ok = s.hip_ok(launch_init_static(L, (uint32_t*)c, NCOUNTERS, (uint32_t*)s.ws.pair_ub.p,
                                                  (uint64_t*)s.ws.pair_d2.p, (uint64_t*)s.ws.pair_tie.p,
                                                  (int32_t*)s.ws.pair_cnt.p, pc), "init") &&
                      (!cluster ||
                       s.hip_ok(launch_broad_phase(L, (const int32_t*)bp.pid.p,
                                                   (const int32_t*)((const char*)bp.pid.p + PAIR_HDR), mcap,
                                                   (const int32_t*)bp.seg.p, seg_cap, (const PartDev*)dpart.p,
                                                   dpart_cap, (const MeshDev*)dmesh.p, (int32_t)meshes.size(), 0.0,
                                                   (BpMember*)bp.mem.p, (int32_t*)bp.row_cnt.p, (int64_t*)bp.row_off.p,
                                                   (int64_t*)bp.seg_pairs.p, (int32_t*)s.ws.dlist.p,
                                                   (int32_t*)dlist, nullptr, pc, c, 29, 18),
                                "broad phase")) &&
                      (!dev || s.hip_ok(launch_pair_gather(L, nlist, dlist, pc, (const PartDev*)dpart.p, dpart_cap,
                                                           (const MeshDev*)dmesh.p, (int32_t)meshes.size(), 0.0, 0, 1,
                                                           item_cap, word_cap, (int32_t*)s.ws.src.p, src_dev(s.ws),
                                                           (int64_t*)s.ws.gather_tmp.p, c, 29, 11, 15, 16),
                                        "pair gather")) &&
                      s.hip_ok(launch_pair_prep(L, (const int32_t*)s.ws.src.p, src_dev(s.ws), pc, popt,
                                                (int32_t*)s.ws.pairs.p, dp, q.tkey, q.tval, q.tmode), "pair prep") &&
                      s.hip_ok(launch_cull(L, dp, nq, pc, S, dense ? 1 : 0, (Item*)s.ws.items.p, (NearItem*)s.ws.items.p,
                                           c + 0, item_cap,
                                           c64 + 4, (int32_t*)s.ws.scan.p, (uint64_t*)s.ws.cullmask.p,
                                           dense ? nullptr : sl + 7 * STAT_WAVES), "cull") &&
                      mark(5);
            if (ok && !dense) {
                ok = s.hip_ok(launch_near(L, dp, S, (const NearItem*)s.ws.items.p, c + 0, item_cap, c + 64, nr, c + 6, nc,
                                          sl, sl + 4 * STAT_WAVES, gnear), "near") &&
                     mark(6) && mark(2) &&
                     s.hip_ok(launch_eval(L, fp64, dp, S, nr, c + 6, nc, (Cand*)s.ws.cands.p, c + 1, cc,
                                          sl + STAT_WAVES, geval), "eval") &&
                     mark(3);
            } else if (ok && !fp64) {
                ok = mark(2) &&
                     s.hip_ok(launch_dist32(L, dp, S, (Item*)s.ws.items.p, c + 0, item_cap, (PartialF*)s.ws.part32.p,
                                            (uint32_t*)s.ws.pair_ub.p, (Cand*)s.ws.cands.p, c + 1, cc, c + 4,
                                            sl + STAT_WAVES, grid32), "dist32") &&
                     mark(3) &&
                     s.hip_ok(launch_refine_select(L, dp, (Item*)s.ws.items.p, c + 0, item_cap, (PartialF*)s.ws.part32.p,
                                                   (uint32_t*)s.ws.pair_ub.p, 1, (Item*)s.ws.refs.p, c + 2, item_cap), "refine") &&
                     s.hip_ok(launch_dist64(L, dp, S, (Item*)s.ws.refs.p, c + 2, item_cap, (PartialD*)s.ws.part64.p,
                                            (uint64_t*)s.ws.pair_d2.p, nullptr, c + 1, 0, c + 5, 0,
                                            sl + 2 * STAT_WAVES, grid64), "dist64");
            } else if (ok) {
                ok = mark(2) &&
                     s.hip_ok(launch_dist64(L, dp, S, (Item*)s.ws.items.p, c + 0, item_cap, (PartialD*)s.ws.part64.p,
                                            (uint64_t*)s.ws.pair_d2.p, (Cand*)s.ws.cands.p, c + 1, cc, c + 5, 1,
                                            sl + STAT_WAVES, grid64), "dist64") &&
                     mark(3);
            }
            ok = ok && s.hip_ok(launch_recheck(L, dp, S, (Cand*)s.ws.cands.p, c + 1, cc, (CandOut*)s.ws.outs.p,
                                               (uint64_t*)s.ws.ckey.p, (uint64_t*)s.ws.cd2.p, (uint64_t*)s.ws.pair_d2.p,
                                               (int32_t*)s.ws.pair_cnt.p,
                                               sl + 3 * STAT_WAVES, sl + 5 * STAT_WAVES, sl + 6 * STAT_WAVES,
                                               (uint32_t*)(c + 34)), "recheck") &&
                      s.hip_ok(launch_pair_scan(L, nq, (int32_t*)s.ws.pair_cnt.p, (int32_t*)s.ws.pair_off.p, c + 20,
                                                (int32_t*)s.ws.large.p),
                               "scan");
            if (ok && dense)
                ok = s.hip_ok(launch_tie(L, ties, tie_count, item_cap, (PartialD*)s.ws.part64.p,
                                         (uint64_t*)s.ws.pair_d2.p, (uint64_t*)s.ws.pair_tie.p), "tie");
            return ok && s.hip_ok(launch_tie_out(L, (uint64_t*)s.ws.ckey.p, (uint64_t*)s.ws.cd2.p, c + 1, cc,
                                                 (uint64_t*)s.ws.pair_d2.p,
                                                 (uint64_t*)s.ws.pair_tie.p), "tie") &&
                   s.hip_ok(launch_pair_final(L, dp, nq, pc, S, (uint64_t*)s.ws.pair_d2.p, (uint64_t*)s.ws.pair_tie.p,
                                              dense ? 1 : 0, (PairOut*)s.ws.pair_out.p), "final") &&
                   s.hip_ok(launch_stat_reduce(L, (const uint64_t*)sl, plan, c64), "counters");
        };
        bool ok = (cluster || q.staged) ? true
                  : dev ? s.hip_ok(hipMemcpyAsync(s.ws.dlist.p, s.ws.h_src.p, sizeof(int32_t), hipMemcpyHostToDevice,
                                                s.stream), "pair count upload") &&
                            s.hip_ok(hipMemcpyAsync((char*)s.ws.dlist.p + PAIR_HDR, q.d_list,
                                                    sizeof(int32_t) * 2 * (size_t)n, hipMemcpyDeviceToDevice,
                                                    s.stream), "pair list copy")
                      : s.hip_ok(hipMemcpyAsync(s.ws.src.p, s.ws.h_src.p, PAIR_HDR + sizeof(PairSrc) * n,
                                                hipMemcpyHostToDevice, s.stream), "pairs upload");
        ok = ok && s.hip_ok(hipEventRecord(ev[0], s.stream), "event");
        if (ok && !timing && use_graphs) {
            const std::vector<uint64_t> key = {
                (uint64_t)cluster, (uint64_t)bp.pid.p, (uint64_t)bp.seg.p, (uint64_t)bp.mem.p, (uint64_t)bp.row_cnt.p,
                (uint64_t)bp.row_off.p, (uint64_t)bp.seg_pairs.p, (uint64_t)mcap, (uint64_t)seg_cap,
                (uint64_t)dev, (uint64_t)s.ws.dlist.p, (uint64_t)s.ws.gather_tmp.p, (uint64_t)dpart.p,
                (uint64_t)dpart_cap, (uint64_t)dmesh.p, (uint64_t)meshes.size(), (uint64_t)word_cap,
                (uint64_t)fp64, (uint64_t)dense, (uint64_t)pc, (uint64_t)item_cap, (uint64_t)cc, (uint64_t)nc,
                (uint64_t)s.ws.src.p, dbits(popt.dt), dbits(popt.tol_rel),
                dbits(popt.margin_c), (uint64_t)popt.samples, (uint64_t)popt.flags,
                (uint64_t)gnear, (uint64_t)geval, (uint64_t)grid32, (uint64_t)grid64,
                (uint64_t)s.ws.pairs.p, (uint64_t)s.ws.items.p, (uint64_t)s.ws.refs.p, (uint64_t)s.ws.part32.p,
                (uint64_t)s.ws.part64.p, (uint64_t)s.ws.near.p, (uint64_t)s.ws.cands.p, (uint64_t)s.ws.outs.p,
                (uint64_t)s.ws.pair_ub.p, (uint64_t)s.ws.pair_d2.p, (uint64_t)s.ws.pair_tie.p,
                (uint64_t)s.ws.pair_out.p, (uint64_t)s.ws.counters.p, (uint64_t)s.ws.scan.p, (uint64_t)s.ws.stats.p,
                (uint64_t)s.ws.pair_cnt.p, (uint64_t)s.ws.pair_off.p, (uint64_t)s.ws.ckey.p, (uint64_t)s.ws.cd2.p,
                (uint64_t)s.ws.large.p,
                (uint64_t)s.ws.cullmask.p,
                (uint64_t)S.v32, (uint64_t)S.v64, (uint64_t)S.orig, (uint64_t)S.pos, (uint64_t)S.tile_sph,
                (uint64_t)S.tri_sph, (uint64_t)S.cap, (uint64_t)q.staged, (uint64_t)q.tkey, (uint64_t)q.tval,
                (uint64_t)q.tmode};
            bool ran = false;
            ok = replay(s, key, true, [&] { return chain(false); }, ran);
            if (ok && !ran) ok = chain(false);
        } else if (ok) {
            ok = chain(timing);
        }
        ok = ok && s.hip_ok(hipEventRecord(ev[1], s.stream), "event") && (!q.before_sync || q.before_sync()) &&
             s.hip_ok(hipMemcpyAsync(s.ws.h_counters.p, c, 64 * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream), "readback") &&
             (cluster || s.hip_ok(hipMemcpyAsync(s.ws.h_pair_out.p, s.ws.pair_out.p, sizeof(PairOut) * n,
                                                 hipMemcpyDeviceToHost, s.stream), "readback")) &&
             (!dev || cluster || s.hip_ok(hipMemcpyAsync(q.pairs.data(), dlist, sizeof(int32_t) * 2 * (size_t)n,
                                                         hipMemcpyDeviceToHost, s.stream), "readback")) &&
             s.hip_ok(hipStreamSynchronize(s.stream), "query");
        if (!ok) return MCD_E_HIP;
        const int32_t* hc = (const int32_t*)s.ws.h_counters.p;
        const int64_t* hc64 = (const int64_t*)hc;
        if (dev) {
            const int32_t gerr = hc[29];
            q.tile_pairs_total = hc64[15];
            q.tri_pairs_covered = hc64[16];
            q.stats.tile_pairs_total = q.tile_pairs_total;
            q.stats.tri_pairs_covered = q.tri_pairs_covered;
            if (gerr & (GATHER_BAD_ID | GATHER_DEAD_MESH)) {
                e = (gerr & GATHER_BAD_ID) ? "query_pairs_dev: unknown particle id (or an id >= 2^24) in the pair list"
                                           : "query_pairs_dev: a pair uses an unloaded mesh";
                return MCD_E_NOT_FOUND;
            }
            if (gerr & GATHER_SAME) { e = "query_pairs_dev: a pair repeats a particle"; return MCD_E_INVALID; }
            if (cluster && hc64[18] > pc) {   // more candidate pairs than the list holds
                q.n_dev = (int32_t)std::min<int64_t>(hc64[18], INT32_MAX);
                q.stats.retries++;
                continue;
            }
            if (gerr & GATHER_OVERFLOW) {   // larger item buffers for the counted tile pairs
                q.stats.retries++;
                continue;
            }
            if (cluster) {
                // the pairs found, their results and each segment's first pair
                n = (int32_t)hc64[18];
                const int32_t nseg = (int32_t)q.seg_off.size() - 1;
                q.pairs.resize(2 * (size_t)n);
                q.seg_pairs.resize(nseg + 1);
                if ((st = s.ws.h_pair_out.reserve(sizeof(PairOut) * std::max(n, 1), e)) != MCD_OK) return st;
                if (!s.hip_ok(hipMemcpyAsync(s.ws.h_pair_out.p, s.ws.pair_out.p, sizeof(PairOut) * n,
                                             hipMemcpyDeviceToHost, s.stream), "readback") ||
                    !s.hip_ok(hipMemcpyAsync(q.pairs.data(), dlist, sizeof(int32_t) * 2 * (size_t)n,
                                             hipMemcpyDeviceToHost, s.stream), "readback") ||
                    !s.hip_ok(hipMemcpyAsync(q.seg_pairs.data(), bp.seg_pairs.p, sizeof(int64_t) * (nseg + 1),
                                             hipMemcpyDeviceToHost, s.stream), "readback") ||
                    !s.hip_ok(hipStreamSynchronize(s.stream), "query"))
                    return MCD_E_HIP;
                if (n == 0) {
                    q.result.clear();
                    q.ncon = 0;
                    return MCD_OK;
                }
            }
        }
        const int64_t ncand = hc[1], nnear = dense ? 0 : hc[6];
        const int64_t nout = hc64[8];   // contacts among the candidates
        if (ncand > cc || nnear > nc) {
            if (ncand > cc) s.cand_cap = (int32_t)std::min<int64_t>(ncand * 2, (int64_t)1 << 30);
            if (nnear > nc) s.near_cap = std::min<int64_t>(nnear + nnear / 2, (int64_t)1 << 31);
            q.stats.retries++;
            continue;
        }
        float ms = 0, mk = 0, mc = 0, mn = 0;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (timing) {
            (void)hipEventElapsedTime(&mk, ev[2], ev[3]);
            (void)hipEventElapsedTime(&mc, ev[0], ev[5]);
            if (!dense) (void)hipEventElapsedTime(&mn, ev[5], ev[6]);
        }
        if (measure) report_shape(bucket, shape, mn + mk);
        q.stats.gpu_ms = ms;
        q.stats.main_ms = mk;
        q.stats.cull_ms = mc;
        q.stats.near_ms = mn;
        q.stats.sort_ms = 0;
        q.stats.tile_pairs_kept = hc[0];
        q.stats.tri_pairs_tiled = hc64[4];
        q.stats.tri_pairs_evaluated = hc64[5];   // full evaluations (dense: every pair of the items)
        q.stats.near_pairs = dense ? 0 : hc64[9];   // sphere-near pairs (the list holds their plane survivors)
        q.stats.sphere_tests = dense ? 0 : hc64[7];
        q.stats.fp64_rechecks = ncand;
        q.stats.refine_items = (fp64 || !dense) ? 0 : hc[2];
        q.stats.banded = hc64[12];
        q.stats.cull_tests = dense ? 0 : hc64[19];
        q.stats.validated = hc64[13];
        {
            float r[2];
            std::memcpy(r, hc + 34, sizeof r);
            q.stats.margin_ratio = r[0];
            q.stats.margin_ratio_np = r[1];
        }
        q.stats.tune_pending = tune_pending(bucket);
        const bool want_contacts = (q.opts.flags & MCD_Q_CONTACTS) != 0;
        const bool devout = (q.opts.flags & MCD_Q_DEVICE_OUT) != 0;
        int64_t fused_count = -1;
        const mcd_contact* dret = nullptr;   // MCD_Q_DEVICE_OUT: the records kept on the device
        // results: contacts sorted by (pair, tri_a, tri_b) on the device; per
        // pair segments sorted in LDS when every pair has at most SEG_CAP
        // contacts, else one radix sort over all records
        if (nout > 0 && want_contacts) {
            const int32_t maxseg = hc[20];
            const bool by_pair = maxseg >= 1 && maxseg <= SEG_CAP;
            size_t tb = 0;
            int pair_bits = 1, tri_bits = 1;
            if (!by_pair) {
                // key widths: the largest pair index and triangle index of the query
                int32_t maxnt = 1;
                for (const MeshInfo& m : (dev ? meshes : q.mi)) maxnt = std::max(maxnt, m.nt);
                while (pair_bits < 31 && ((int64_t)1 << pair_bits) < n) ++pair_bits;
                while (tri_bits < 16 && ((int64_t)1 << tri_bits) < maxnt) ++tri_bits;
                if (!s.hip_ok(sort_contacts(L, nullptr, (int32_t)ncand, (int32_t)nout, pair_bits, tri_bits, nullptr,
                                            nullptr, nullptr, nullptr, nullptr, tb, nullptr), "sort"))
                    return MCD_E_HIP;
                if ((st = s.ws.keys.reserve(sizeof(uint64_t) * 2 * ncand, e)) != MCD_OK ||
                    (st = s.ws.idx.reserve(sizeof(int32_t) * 2 * ncand, e)) != MCD_OK ||
                    (st = s.ws.sort_tmp.reserve(tb, e)) != MCD_OK)
                    return st;
            }
            if ((st = s.ws.sorted.reserve(sizeof(mcd_contact) * nout, e)) != MCD_OK) return st;
            if (!devout) {
                if (q.cpin) { pinned.put(q.cpin); q.cpin = nullptr; }
                q.pool = &pinned;
                q.cpin = pinned.get(sizeof(mcd_contact) * nout, e);
                if (!q.cpin) return MCD_E_OOM;
            }
            bool oks = s.hip_ok(hipEventRecord(ev[4], s.stream), "event");
            if (by_pair) {
                int p2 = 1;
                while (p2 < maxseg) p2 <<= 1;
                oks = oks && s.hip_ok(sort_contacts_by_pair(L, (CandOut*)s.ws.outs.p, (uint64_t*)s.ws.ckey.p,
                                                            (int32_t)ncand, n,
                                                            (int32_t*)s.ws.pair_off.p, (int32_t*)s.ws.pair_cnt.p,
                                                            (const int32_t*)s.ws.large.p, std::min(hc[21], n),
                                                            (uint64_t*)s.ws.seg.p, p2, (mcd_contact*)s.ws.sorted.p),
                                      "sort");
            } else {
                uint64_t* keys = (uint64_t*)s.ws.keys.p;
                int32_t* idx = (int32_t*)s.ws.idx.p;
                tb = s.ws.sort_tmp.bytes;
                oks = oks && s.hip_ok(sort_contacts(L, (CandOut*)s.ws.outs.p, (int32_t)ncand, (int32_t)nout, pair_bits,
                                                    tri_bits, keys, keys + ncand, idx, idx + ncand, s.ws.sort_tmp.p, tb,
                                                    (mcd_contact*)s.ws.sorted.p), "sort");
            }
            int64_t nret = nout;
            const mcd_contact* ret = (const mcd_contact*)s.ws.sorted.p;
            if (oks && (q.opts.flags & MCD_Q_FUSE)) {
                // contact fusion per pair over the sorted records, then the
                // groups gathered: one more round trip for their count
                if ((st = s.ws.goff.reserve(sizeof(int32_t) * ((size_t)n + 1), e)) != MCD_OK ||
                    (st = s.ws.fused.reserve(sizeof(mcd_contact) * nout, e)) != MCD_OK)
                    return st;
                oks = s.hip_ok(launch_fuse(L, dp, nq, n, (const int32_t*)s.ws.pair_off.p, (mcd_contact*)s.ws.sorted.p,
                                           (int32_t*)s.ws.seg.p, (int32_t*)s.ws.pair_cnt.p), "fuse") &&
                      s.hip_ok(launch_pair_scan(L, nq, (const int32_t*)s.ws.pair_cnt.p, (int32_t*)s.ws.goff.p, c + 20,
                                                (int32_t*)s.ws.large.p), "fuse") &&
                      s.hip_ok(launch_fuse_gather(L, nq, n, (const int32_t*)s.ws.pair_off.p,
                                                  (const int32_t*)s.ws.goff.p, (const mcd_contact*)s.ws.sorted.p,
                                                  (mcd_contact*)s.ws.fused.p), "fuse");
                int32_t tot = 0;
                oks = oks && s.hip_ok(hipMemcpyAsync(&tot, (int32_t*)s.ws.goff.p + n, sizeof(int32_t),
                                                     hipMemcpyDeviceToHost, s.stream), "readback") &&
                      s.hip_ok(hipStreamSynchronize(s.stream), "query");
                nret = tot;
                ret = (const mcd_contact*)s.ws.fused.p;
            }
            if (!oks || !s.hip_ok(hipEventRecord(ev[7], s.stream), "event") ||
                (!devout && (!s.hip_ok(hipMemcpyAsync(q.cpin->p, ret, sizeof(mcd_contact) * nret,
                                                      hipMemcpyDeviceToHost, s.stream), "readback") ||
                             !s.hip_ok(hipStreamSynchronize(s.stream), "query"))))
                return MCD_E_HIP;
            fused_count = nret;
            dret = ret;
            if (!devout) {
                float so = 0;
                (void)hipEventElapsedTime(&so, ev[4], ev[7]);
                q.stats.sort_ms = so;
                q.stats.gpu_ms += so;
            }
        }
        if (devout) {
            // pair results and contact records copied on the device into a
            // buffer the ticket holds (no host copy of the records)
            const int64_t nk = fused_count > 0 ? fused_count : 0;
            const size_t pbytes = (sizeof(mcd_pair_result) * (size_t)n + 255) / 256 * 256;
            if (q.dout) { devpool.put(q.dout); q.dout = nullptr; }
            q.dpool = &devpool;
            q.dout = devpool.get(pbytes + sizeof(mcd_contact) * (size_t)nk, e);
            if (!q.dout) return MCD_E_OOM;
            q.dout_con = pbytes;
            if ((!q.dev_done && !s.hip_ok(hipEventCreateWithFlags(&q.dev_done, hipEventDisableTiming), "event")) ||
                (n > 0 && !s.hip_ok(hipMemcpyAsync(q.dout->p, s.ws.pair_out.p, sizeof(PairOut) * (size_t)n,
                                                   hipMemcpyDeviceToDevice, s.stream), "device results")) ||
                (nk > 0 && !s.hip_ok(hipMemcpyAsync((char*)q.dout->p + pbytes, dret, sizeof(mcd_contact) * (size_t)nk,
                                                    hipMemcpyDeviceToDevice, s.stream), "device results")) ||
                !s.hip_ok(hipEventRecord(q.dev_done, s.stream), "event") ||
                !s.hip_ok(hipEventSynchronize(q.dev_done), "query"))
                return MCD_E_HIP;
            if (nk > 0) {
                float so = 0;
                (void)hipEventElapsedTime(&so, ev[4], ev[7]);
                q.stats.sort_ms = so;
                q.stats.gpu_ms += so;
            }
        }
        const PairOut* po = (const PairOut*)s.ws.h_pair_out.p;
        const bool want_closest = (q.opts.flags & MCD_Q_CLOSEST) != 0;
        q.result.resize(n);
        for (int i = 0; i < n; ++i) {
            mcd_pair_result& r = q.result[i];
            r.dmin = want_closest ? po[i].d : INFINITY;
            for (int k = 0; k < 3; ++k) {
                r.pa[k] = want_closest ? po[i].pa[k] : 0.0;
                r.pb[k] = want_closest ? po[i].pb[k] : 0.0;
            }
            r.toi = 0.0;
            r.tri_a = want_closest ? po[i].tri_a : -1;
            r.tri_b = want_closest ? po[i].tri_b : -1;
            r.contact = po[i].contact;
            r.status = po[i].contact;
        }
        q.ncon = want_contacts ? (fused_count >= 0 ? fused_count : nout) : 0;
        return MCD_OK;
    }
    s.err = "query: buffer regrow did not converge";
    return MCD_E_OOM;
}

// Replay the captured chain of `key`, capturing it first if needed. With
// capture_first false a key is captured only when it is met the second
// time (queries of changing shape then run eagerly instead of capturing a
// graph each time). ran: whether the chain was launched (replayed, or
// captured and replayed); false leaves the eager launch to the caller.
bool Ctx::replay(Slot& s, const std::vector<uint64_t>& key, bool capture_first, const std::function<bool()>& chain,
                 bool& ran)
{
    ran = false;
    hipGraphExec_t exec = nullptr;
    for (auto& g : s.graphs)
        if (g.key == key) { exec = g.exec; g.used = ++s.graph_clock; break; }
    if (!exec) {
        if (!capture_first) {
            if (s.seen.size() > 64) s.seen.clear();
            if (++s.seen[key] < 2) return true;
        }
        hipGraph_t g = nullptr;
        bool ok = s.hip_ok(hipStreamBeginCapture(s.stream, hipStreamCaptureModeRelaxed), "graph capture");
        if (!ok) return false;
        const bool okc = chain();
        const hipError_t ee = hipStreamEndCapture(s.stream, &g);
        ok = okc && s.hip_ok(ee, "graph capture") && s.hip_ok(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0),
                                                              "graph instantiate");
        if (g) (void)hipGraphDestroy(g);
        if (!ok) return false;
        ++graph_captures;
        if ((int)s.graphs.size() >= MAX_GRAPHS) {
            auto lru = std::min_element(s.graphs.begin(), s.graphs.end(),
                                        [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
            (void)hipGraphExecDestroy(lru->exec);
            s.graphs.erase(lru);
        }
        s.graphs.push_back(GraphEntry{key, exec, ++s.graph_clock});
    }
    ran = true;
    return s.hip_ok(hipGraphLaunch(exec, s.stream), "graph launch");
}

// The paper's narrowing estimate: every tile pair of the query (dense cull),
// rounds until no pair's span narrows any further, then the triangle pair
// in contact at each pair's final time. keys/times as phase 1 of run_toi
// gives them: no contact -> ~0; else (status part << 32) | (i << 16 | j).
mcd_status Ctx::run_narrow(Query& q, Slot& s, std::vector<uint64_t>& keys, std::vector<double>& times)
{
    const int32_t n = (int32_t)q.src.size();
    const int32_t nn = std::max(n, 1);
    Launch L{s.stream, num_cu};
    std::string& e = s.err;
    mcd_status st;
    const int64_t item_cap = std::max<int64_t>(1, q.tile_pairs_total);
    if ((st = s.ws.pairs.reserve(PAIR_HDR + sizeof(PairDev) * nn, e)) != MCD_OK ||
        (st = s.ws.items.reserve(sizeof(Item) * item_cap, e)) != MCD_OK ||
        (st = s.ws.scan.reserve(cull_scan_bytes(nn), e)) != MCD_OK ||
        (st = s.ws.cullmask.reserve(sizeof(uint64_t) * ((size_t)item_cap / 64 + nn + 1), e)) != MCD_OK ||
        (st = s.ws.pair_t.reserve(sizeof(double) * nn, e)) != MCD_OK ||
        (st = s.ws.pair_key.reserve(sizeof(uint64_t) * nn, e)) != MCD_OK ||
        (st = s.ws.pair_kub.reserve(sizeof(uint32_t) * nn, e)) != MCD_OK ||
        (st = s.ws.pair_cnt.reserve(sizeof(int32_t) * nn, e)) != MCD_OK ||
        (st = s.ws.counters.reserve(sizeof(int32_t) * NCOUNTERS, e)) != MCD_OK ||
        (st = s.ws.stats.reserve(sizeof(uint64_t) * STAT_ROWS * STAT_WAVES, e)) != MCD_OK ||
        (st = s.ws.h_counters.reserve(sizeof(int32_t) * 64, e)) != MCD_OK ||
        (st = s.ws.h_key.reserve(sizeof(uint64_t) * nn, e)) != MCD_OK ||
        (st = s.ws.h_t.reserve(sizeof(double) * nn, e)) != MCD_OK ||
        (st = s.ws.h_ij.reserve(2 * sizeof(int32_t) * nn, e)) != MCD_OK)
        return st;
    int64_t nwords = 0;
    if ((st = stage_src(q, s, nn, false, nwords)) != MCD_OK) return st;
    int32_t* c = (int32_t*)s.ws.counters.p;
    unsigned long long* c64 = (unsigned long long*)c;
    unsigned long long* sl = (unsigned long long*)s.ws.stats.p;
    const int32_t* nq = (const int32_t*)s.ws.pairs.p;
    PairDev* dp = pairs_dev(s.ws);
    TriStore S = store();
    double* pT = (double*)s.ws.pair_t.p;
    uint64_t* pnext = (uint64_t*)s.ws.pair_key.p;
    uint32_t* pij = (uint32_t*)s.ws.pair_kub.p;
    int32_t* found = (int32_t*)s.ws.pair_cnt.p;
    const int grid = (int)std::min<int64_t>(num_cu * 16, std::max<int64_t>(1, q.tile_pairs_total));
    const StatPlan plan{1, {grid}, {12}};
    // counters: 0 items, 40 the round's change flag, 8-9 tiled triangle
    // pairs, 24-25 triangle-pair evaluations (all rounds)
    bool ok = s.hip_ok(hipMemcpyAsync(s.ws.src.p, s.ws.h_src.p, PAIR_HDR + sizeof(PairSrc) * n,
                                      hipMemcpyHostToDevice, s.stream), "pairs upload") &&
              s.hip_ok(hipEventRecord(s.ev[0], s.stream), "event") &&
              s.hip_ok(launch_fill_u32(L, (uint32_t*)c, NCOUNTERS, 0), "fill") &&
              s.hip_ok(launch_pair_prep(L, (const int32_t*)s.ws.src.p, src_dev(s.ws), nn, prep_opts(q.opts),
                                        (int32_t*)s.ws.pairs.p, dp), "pair prep") &&
              s.hip_ok(launch_cull(L, dp, nq, nn, S, 1, (Item*)s.ws.items.p, nullptr, c + 0, item_cap, c64 + 4,
                                   (int32_t*)s.ws.scan.p, (uint64_t*)s.ws.cullmask.p), "cull") &&
              s.hip_ok(launch_narrow_init(L, nq, nn, dp, pT, pnext, pij, found), "narrowing");
    if (!ok) return MCD_E_HIP;
    int32_t* hc = (int32_t*)s.ws.h_counters.p;
    int rounds = 0;
    for (rounds = 1; rounds <= 200; ++rounds) {
        ok = s.hip_ok(launch_fill_u32(L, (uint32_t*)(c + 40), 1, 0), "narrowing") &&
             s.hip_ok(launch_narrow_round(L, dp, S, (const Item*)s.ws.items.p, c + 0, item_cap, pT, pnext, pij, 0,
                                          sl, grid), "narrowing") &&
             s.hip_ok(launch_stat_reduce(L, (const uint64_t*)sl, plan, c64), "counters") &&
             s.hip_ok(launch_narrow_update(L, nq, nn, pT, pnext, found, c + 40), "narrowing") &&
             s.hip_ok(hipMemcpyAsync(hc + 40, c + 40, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream), "readback") &&
             s.hip_ok(hipStreamSynchronize(s.stream), "narrowing");
        if (!ok) return MCD_E_HIP;
        if (hc[40] == 0) break;
    }
    ok = s.hip_ok(launch_narrow_round(L, dp, S, (const Item*)s.ws.items.p, c + 0, item_cap, pT, pnext, pij, 1, sl,
                                      grid), "narrowing") &&
         s.hip_ok(launch_stat_reduce(L, (const uint64_t*)sl, plan, c64), "counters") &&
         s.hip_ok(hipEventRecord(s.ev[1], s.stream), "event") &&
         s.hip_ok(hipMemcpyAsync(hc, c, 32 * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream), "readback") &&
         s.hip_ok(hipMemcpyAsync(s.ws.h_t.p, pT, sizeof(double) * n, hipMemcpyDeviceToHost, s.stream), "readback") &&
         s.hip_ok(hipMemcpyAsync(s.ws.h_key.p, pij, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s.stream),
                  "readback") &&
         s.hip_ok(hipMemcpyAsync(s.ws.h_ij.p, found, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s.stream),
                  "readback") &&
         s.hip_ok(hipStreamSynchronize(s.stream), "narrowing");
    if (!ok) return MCD_E_HIP;
    const double* hT = (const double*)s.ws.h_t.p;
    const uint32_t* hij = (const uint32_t*)s.ws.h_key.p;
    const int32_t* hf = (const int32_t*)s.ws.h_ij.p;
    keys.assign(n, ~0ull);
    times.assign(n, INFINITY);
    for (int i = 0; i < n; ++i) {
        if (!hf[i] || hij[i] == 0xffffffffu) continue;
        times[i] = hT[i];
        keys[i] = ((uint64_t)(hT[i] == 0.0 ? 0 : 1) << 32) | hij[i];
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, s.ev[0], s.ev[1]);
    q.stats.gpu_ms = ms;
    q.stats.main_ms = ms;
    q.stats.tile_pairs_total = q.tile_pairs_total;
    q.stats.tile_pairs_kept = hc[0];
    q.stats.tri_pairs_covered = q.tri_pairs_covered;
    q.stats.tri_pairs_tiled = *(const int64_t*)(hc + 8);
    q.stats.fp64_evals = *(const int64_t*)(hc + 24);
    q.stats.candidates = rounds;
    return MCD_OK;
}

mcd_status Ctx::run_toi(Query& q, Slot& s)
{
    if (q.dev && q.src.empty() && q.n_dev > 0) {
        // Time stamps from a device pair list, or from a cluster's pairs found
        // on the device: the list is read back once it is ready and the pairs
        // are snapshot from the host tables, which no call can change while
        // this query is in flight (see wait_no_readers).
        std::vector<int32_t> h;
        if (q.cluster) {
            std::vector<int64_t> seg;
            mcd_status st = s.ws.counters.reserve(sizeof(int32_t) * NCOUNTERS, s.err);
            if (st == MCD_OK)
                st = broad_phase_eager(s.ws.bp, s.stream, (int32_t*)s.ws.counters.p, q.members, q.seg_off,
                                       q.opts.dt, s.ws.dlist, false, h, seg, s.err);
            if (st != MCD_OK) return st;
        } else {
            h.resize(2 * (size_t)q.n_dev);
            if (!s.hip_ok(hipStreamWaitEvent(s.stream, q.ready, 0), "wait for the pair list") ||
                !s.hip_ok(hipMemcpyAsync(h.data(), q.d_list, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                                         s.stream), "pair list read") ||
                !s.hip_ok(hipStreamSynchronize(s.stream), "pair list read"))
                return MCD_E_HIP;
        }
        mcd_status st = prepare_pairs(h.data(), (int32_t)(h.size() / 2), q, s.err);
        if (st != MCD_OK) return st;
        q.stats.tile_pairs_total = q.tile_pairs_total;
        q.stats.tri_pairs_covered = q.tri_pairs_covered;
    }
    const int32_t n = (int32_t)q.src.size();
    const bool narrow = (q.opts.flags & MCD_Q_NARROW) != 0;
    const int Sn = q.opts.samples, rows = Sn + 1;
    const bool fp64 = (q.opts.flags & MCD_Q_FP64) != 0;
    Launch L{s.stream, num_cu};
    std::string& e = s.err;
    mcd_status st;
    const int64_t item_cap = std::max<int64_t>(1, q.tile_pairs_total);
    const int nn = std::max(n, 1);
    if (n == 0) {
        q.result.clear();
        q.ncon = 0;
        return MCD_OK;
    }
    hipEvent_t* tev = s.ev + 8;   // the first phase's events
    if (narrow) {
        // the narrowing's time stamps, on the device for the second phase
        std::vector<uint64_t> keys;
        std::vector<double> times;
        if ((st = run_narrow(q, s, keys, times)) != MCD_OK) return st;
        if ((st = s.ws.pair_key.reserve(sizeof(uint64_t) * nn, e)) != MCD_OK ||
            (st = s.ws.pair_t.reserve(sizeof(double) * nn, e)) != MCD_OK ||
            (st = s.ws.h_key.reserve(sizeof(uint64_t) * nn, e)) != MCD_OK ||
            (st = s.ws.h_t.reserve(sizeof(double) * nn, e)) != MCD_OK ||
            (st = s.ws.eval_out.reserve(sizeof(PairOut) * nn, e)) != MCD_OK ||
            (st = s.ws.h_eval.reserve(sizeof(PairOut) * nn, e)) != MCD_OK)
            return st;
        std::memcpy(s.ws.h_key.p, keys.data(), sizeof(uint64_t) * n);
        std::memcpy(s.ws.h_t.p, times.data(), sizeof(double) * n);
        if (!s.hip_ok(hipMemcpyAsync(s.ws.pair_key.p, s.ws.h_key.p, sizeof(uint64_t) * n, hipMemcpyHostToDevice,
                                     s.stream), "upload") ||
            !s.hip_ok(hipMemcpyAsync(s.ws.pair_t.p, s.ws.h_t.p, sizeof(double) * n, hipMemcpyHostToDevice,
                                     s.stream), "upload"))
            return MCD_E_HIP;
    }
    mcd_stats keep = q.stats;
    std::unique_ptr<Query> sub;
    for (int attempt = 0;; ++attempt) {
        bool timing = false;
        int64_t cc = 0, rc = 0, sc = 0;
        if (!narrow) {
            if (attempt >= 8) { s.err = "query: buffer regrow did not converge"; return MCD_E_OOM; }
            cc = s.cand_cap; rc = s.trec_cap; sc = s.srec_cap;
            if ((st = s.ws.pairs.reserve(PAIR_HDR + sizeof(PairDev) * nn, e)) != MCD_OK ||
                (st = s.ws.trecs.reserve(sizeof(ToiRec) * rc, e)) != MCD_OK ||
                (st = s.ws.srecs.reserve(sizeof(ToiRec) * sc, e)) != MCD_OK ||
                (st = s.ws.items.reserve(sizeof(ToiItem) * item_cap, e)) != MCD_OK ||
                (st = s.ws.table.reserve(sizeof(float) * 12 * (size_t)nn * rows, e)) != MCD_OK ||
                (st = s.ws.table64.reserve(sizeof(double) * 12 * (size_t)nn * rows, e)) != MCD_OK ||
                (st = s.ws.eg.reserve(sizeof(Cand) * cc, e)) != MCD_OK ||
                (st = s.ws.eg_out.reserve(sizeof(ToiOut) * cc, e)) != MCD_OK ||
                (st = s.ws.pair_key.reserve(sizeof(uint64_t) * nn, e)) != MCD_OK ||
                (st = s.ws.pair_t.reserve(sizeof(double) * nn, e)) != MCD_OK ||
                (st = s.ws.pair_kub.reserve(sizeof(int32_t) * nn, e)) != MCD_OK ||
                (st = s.ws.counters.reserve(sizeof(int32_t) * NCOUNTERS, e)) != MCD_OK ||
                (st = s.ws.stats.reserve(sizeof(uint64_t) * STAT_ROWS * STAT_WAVES, e)) != MCD_OK ||
                (st = s.ws.h_tcounters.reserve(sizeof(int32_t) * 32, e)) != MCD_OK ||
                (st = s.ws.eval_out.reserve(sizeof(PairOut) * nn, e)) != MCD_OK ||
                (st = s.ws.h_eval.reserve(sizeof(PairOut) * nn, e)) != MCD_OK ||
                (st = s.ws.h_key.reserve(sizeof(uint64_t) * nn, e)) != MCD_OK ||
                (st = s.ws.h_t.reserve(sizeof(double) * nn, e)) != MCD_OK)
                return st;
            // pair sources with the offsets of each pair's tile pairs in the item list
            int64_t ntp = 0;
            if ((st = stage_src(q, s, nn, true, ntp)) != MCD_OK) return st;
            if (ntp > item_cap || ntp > INT32_MAX) { e = "query: too many tile pairs"; return MCD_E_INVALID; }
            PairDev* dp = pairs_dev(s.ws);
            int32_t* c = (int32_t*)s.ws.counters.p;
            TriStore S = store();
            Cand* eg = (Cand*)s.ws.eg.p;
            ToiItem* items = (ToiItem*)s.ws.items.p;
            // per-wave counts: rows 0-3 the sphere stages (gap evaluations of
            // stages 1 and 1b, kept tile pairs, their triangle pairs), row 4 the
            // triangle walk's samples, rows 5-6 the end-game's evaluations and
            // graze leaves
            unsigned long long* sl = (unsigned long long*)s.ws.stats.p;
            const int gsph = num_cu * 16, gwalk = fp64 ? num_cu * 4 : num_cu * 16;
            const int geg = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (cc + 63) / 64));
            const StatPlan plan{7, {gsph, gsph, gsph, gsph, gwalk, geg, geg}, {8, 8, 9, 4, 5, 6, 7}};
            if (gsph > STAT_WAVES || gwalk > STAT_WAVES) { e = "query: grid exceeds the counter slots"; return MCD_E_INVALID; }
            // Phase 1: sample tables, space-time cull, sphere walks, FP32 walk,
            // FP64 end-game, per-pair time stamps. Captured as a graph (no events
            // inside) unless per-stage times are asked for; events 2 / 6 / 3 / 4
            // bracket the stages when they are.
            timing = (q.opts.flags & MCD_Q_TIMING) != 0;
            const PrepOpts popt = prep_opts(q.opts);
            auto chain = [&](bool events) -> bool {
                auto mark = [&](int i) { return !events || s.hip_ok(hipEventRecord(tev[i], s.stream), "event"); };
                return s.hip_ok(launch_pair_prep(L, (const int32_t*)s.ws.src.p, src_dev(s.ws), nn, popt,
                                                 (int32_t*)s.ws.pairs.p, dp), "pair prep") &&
                       s.hip_ok(launch_fill_u32(L, (uint32_t*)c, NCOUNTERS, 0), "fill") &&
                       s.hip_ok(launch_fill_u64(L, (uint64_t*)s.ws.pair_key.p, n, ~0ull), "fill") &&
                       s.hip_ok(launch_fill_u32(L, (uint32_t*)s.ws.pair_kub.p, n, (uint32_t)(Sn + 1)), "fill") &&
                       s.hip_ok(launch_toi_table(L, dp, n, rows, (float*)s.ws.table.p, (double*)s.ws.table64.p), "table") &&
                       s.hip_ok(launch_toi_cull(L, dp, n, S, (float*)s.ws.table.p, items), "toi cull") &&
                       mark(2) &&
                       s.hip_ok(launch_toi_spheres(L, dp, S, (float*)s.ws.table.p, items, ntp, c + 64,
                                                   (int32_t*)s.ws.pair_kub.p, (ToiRec*)s.ws.trecs.p, c + 6, rc,
                                                   (ToiRec*)s.ws.srecs.p, c + 7, sc, sl, gsph), "toi sphere walks") &&
                       mark(6) &&
                       s.hip_ok(launch_toi_walk(L, dp, S, (float*)s.ws.table.p, (double*)s.ws.table64.p, fp64 ? 1 : 0,
                                                (ToiRec*)s.ws.trecs.p, c + 6, rc, c + 64 + 2 * XCD_Q_BLOCK,
                                                (int32_t*)s.ws.pair_kub.p, eg, c + 3, cc, sl + 4 * STAT_WAVES,
                                                gwalk), "toi sampler") &&
                       mark(3) &&
                       s.hip_ok(launch_toi_endgame(L, dp, S, eg, c + 3, cc, (uint64_t*)s.ws.pair_key.p,
                                                   (ToiOut*)s.ws.eg_out.p, sl + 5 * STAT_WAVES, 0, geg), "toi end-game") &&
                       s.hip_ok(launch_toi_final(L, eg, c + 3, cc, (ToiOut*)s.ws.eg_out.p, (uint64_t*)s.ws.pair_key.p,
                                                 (double*)s.ws.pair_t.p), "toi final") &&
                       s.hip_ok(launch_stat_reduce(L, (const uint64_t*)sl, plan, (unsigned long long*)c), "counters") &&
                       mark(4);
            };
            bool ok = s.hip_ok(hipMemcpyAsync(s.ws.src.p, s.ws.h_src.p, PAIR_HDR + sizeof(PairSrc) * n,
                                              hipMemcpyHostToDevice, s.stream), "pairs upload") &&
                      s.hip_ok(hipEventRecord(tev[0], s.stream), "event");
            bool ran = false;
            if (ok && !timing && use_graphs) {
                const std::vector<uint64_t> key = {
                    (uint64_t)n, (uint64_t)nn, (uint64_t)ntp, (uint64_t)rows, (uint64_t)cc, (uint64_t)rc, (uint64_t)sc,
                    (uint64_t)fp64, (uint64_t)gsph, (uint64_t)gwalk, (uint64_t)geg, dbits(popt.dt), dbits(popt.tol_rel),
                    dbits(popt.margin_c), (uint64_t)popt.samples, (uint64_t)popt.flags, (uint64_t)s.ws.src.p,
                    (uint64_t)s.ws.pairs.p, (uint64_t)s.ws.counters.p, (uint64_t)s.ws.pair_key.p, (uint64_t)s.ws.pair_kub.p,
                    (uint64_t)s.ws.pair_t.p, (uint64_t)s.ws.table.p, (uint64_t)s.ws.table64.p, (uint64_t)s.ws.items.p,
                    (uint64_t)s.ws.trecs.p, (uint64_t)s.ws.srecs.p, (uint64_t)s.ws.eg.p, (uint64_t)s.ws.eg_out.p,
                    (uint64_t)s.ws.stats.p, (uint64_t)S.v32, (uint64_t)S.v64, (uint64_t)S.tile_sph, (uint64_t)S.tri_sph,
                    (uint64_t)S.p32, (uint64_t)S.p64, (uint64_t)S.cap, 0x70691ull};
                ok = replay(s, key, false, [&] { return chain(false); }, ran);
            }
            if (ok && !ran) ok = chain(timing);
            // the first phase's results come back with the second phase's
            ok = ok && s.hip_ok(hipEventRecord(tev[1], s.stream), "event") &&
                 s.hip_ok(hipMemcpyAsync(s.ws.h_tcounters.p, c, 32 * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream),
                          "readback") &&
                 s.hip_ok(hipMemcpyAsync(s.ws.h_key.p, s.ws.pair_key.p, sizeof(uint64_t) * n, hipMemcpyDeviceToHost,
                                         s.stream), "readback") &&
                 s.hip_ok(hipMemcpyAsync(s.ws.h_t.p, s.ws.pair_t.p, sizeof(double) * n, hipMemcpyDeviceToHost,
                                         s.stream), "readback");
            if (!ok) return MCD_E_HIP;
        }
        // Phase 2, on the device after phase 1 (no host round trip between
        // them): the static query at each pair's time stamp over the same
        // pair sources (pairs without one have no tile pairs), then the
        // distance and closest points of each pair's winning triangle pair.
        sub.reset(new Query());
        sub->opts = q.opts;
        sub->opts.dt = 0.0;
        sub->opts.flags = ((q.opts.flags & MCD_Q_FP64) ? MCD_Q_FP64 : MCD_Q_MIXED) |
                         (q.opts.flags & (MCD_Q_CONTACTS | MCD_Q_FUSE)) | MCD_Q_CLOSEST;
        sub->staged = true;
        sub->n_dev = n;
        sub->mi = q.mi;
        sub->tile_pairs_total = q.tile_pairs_total;
        sub->tri_pairs_covered = q.tri_pairs_covered;
        sub->tkey = (const uint64_t*)s.ws.pair_key.p;
        sub->tval = (const double*)s.ws.pair_t.p;
        sub->tmode = narrow ? PREP_ZERO_SPIN : PREP_TP0_WORDS;
        // the grids are sized for the pairs with a time stamp, unknown
        // until the query ends: the slot's last time-stamp query's count
        // (first query: a sixteenth of all), which only affects speed
        sub->grid_tile_pairs = s.staged_tp >= 0 ? s.staged_tp : q.tile_pairs_total / 16;
        sub->before_sync = [&]() {
            return s.hip_ok(launch_pair_eval(L, pairs_dev(s.ws), n, store(), nullptr, (PairOut*)s.ws.eval_out.p,
                                             (const uint64_t*)s.ws.pair_key.p), "pair eval") &&
                   s.hip_ok(hipMemcpyAsync(s.ws.h_eval.p, s.ws.eval_out.p, sizeof(PairOut) * n, hipMemcpyDeviceToHost,
                                           s.stream), "readback");
        };
        if ((st = run_static(*sub, s)) != MCD_OK) return st;
        if (narrow) break;
        const int32_t* hc = (const int32_t*)s.ws.h_tcounters.p;
        if (hc[3] > cc || hc[6] > rc || hc[7] > sc) {
            if (hc[3] > cc) s.cand_cap = (int32_t)std::min<int64_t>((int64_t)hc[3] * 2, (int64_t)1 << 30);
            if (hc[6] > rc) s.trec_cap = std::min<int64_t>((int64_t)hc[6] + hc[6] / 2, (int64_t)1 << 31);
            if (hc[7] > sc) s.srec_cap = std::min<int64_t>((int64_t)hc[7] + hc[7] / 2, (int64_t)1 << 31);
            keep.retries++;
            continue;
        }
        float ms = 0, mk = 0, mc = 0, mn = 0, me = 0;
        (void)hipEventElapsedTime(&ms, tev[0], tev[1]);
        if (timing) {
            (void)hipEventElapsedTime(&mc, tev[0], tev[2]);
            (void)hipEventElapsedTime(&mn, tev[2], tev[6]);
            (void)hipEventElapsedTime(&mk, tev[6], tev[3]);
            (void)hipEventElapsedTime(&me, tev[3], tev[4]);
        }
        keep.gpu_ms = ms;
        keep.main_ms = mk;
        keep.cull_ms = mc;
        keep.near_ms = mn;
        keep.endgame_ms = me;
        keep.sphere_tests = *(const int64_t*)(hc + 16);
        keep.tile_pairs_total = q.tile_pairs_total;
        keep.tile_pairs_kept = *(const int64_t*)(hc + 18);
        keep.tri_pairs_covered = q.tri_pairs_covered;
        keep.tri_pairs_tiled = *(const int64_t*)(hc + 8);
        keep.tri_pairs_evaluated = hc[6];   // triangle pairs whose walk starts inside the step
        keep.fp32_samples = *(const int64_t*)(hc + 10);
        keep.candidates = hc[3];
        keep.fp64_rechecks = hc[3];
        keep.fp64_evals = *(const int64_t*)(hc + 12);
        keep.grazes = *(const int64_t*)(hc + 14);
        break;
    }
    keep.retries += sub->stats.retries;
    keep.gpu_ms += sub->stats.gpu_ms;
    q.stats = keep;
    // pair results: the time stamp, and the winning triangle pair's distance
    // and closest points there
    const uint64_t* keys = (const uint64_t*)s.ws.h_key.p;
    const double* times = (const double*)s.ws.h_t.p;
    const PairOut* po = (const PairOut*)s.ws.h_eval.p;
    std::vector<double> tstar(n, INFINITY);
    q.result.assign(n, mcd_pair_result{});
    int64_t keyed_tp = 0;
    for (int i = 0; i < n; ++i) {
        mcd_pair_result& r = q.result[i];
        r.dmin = INFINITY;
        r.toi = INFINITY;
        r.tri_a = r.tri_b = -1;
        r.contact = 0;
        r.status = MCD_NONE;
        if (keys[i] == ~0ull) continue;
        keyed_tp += (int64_t)q.src[i].nta * q.src[i].ntb;
        tstar[i] = (keys[i] >> 32) == 0 ? 0.0 : times[i];
        r.dmin = po[i].d;
        for (int j = 0; j < 3; ++j) { r.pa[j] = po[i].pa[j]; r.pb[j] = po[i].pb[j]; }
        r.tri_a = po[i].tri_a;
        r.tri_b = po[i].tri_b;
        r.toi = tstar[i];
        r.contact = 1;
        r.status = (keys[i] >> 32) == 0 ? MCD_AT_START : MCD_COLLIDES;
    }
    s.staged_tp = keyed_tp;
    // contact records at each pair's time stamp (pair indices are the query's)
    if (q.cpin) { pinned.put(q.cpin); q.cpin = nullptr; }
    q.pool = &pinned;
    q.cpin = sub->cpin;
    sub->cpin = nullptr;
    q.cvec = std::move(sub->cvec);
    q.ncon = sub->ncon;
    mcd_contact* cd = q.cdata();
    for (int64_t k = 0; k < q.ncon; ++k) cd[k].t = tstar[cd[k].pair];
    if (!(q.opts.flags & MCD_Q_CLOSEST))
        for (auto& r : q.result) {
            r.dmin = INFINITY;
            r.tri_a = r.tri_b = -1;
            for (int k = 0; k < 3; ++k) r.pa[k] = r.pb[k] = 0.0;
        }
    return MCD_OK;
}


// The autotuner's table on disk: a header line naming the format, the device
// model and the launch shapes, then one line per tuned bucket (bucket, best
// shape). Anything that does not match is ignored.
static std::string tune_header(const std::string& dev)
{
    std::string h = "mcd-tune 1 " + dev + " shapes";
    for (const Shape& sh : kShapes) h += " " + std::to_string(sh.near_wpc) + "/" + std::to_string(sh.eval_wpc);
    return h;
}

void Ctx::tune_load()
{
    if (tune_path.empty()) return;
    FILE* f = std::fopen(tune_path.c_str(), "r");
    if (!f) return;
    char line[1024];
    bool ok = std::fgets(line, sizeof line, f) != nullptr;
    if (ok) {
        std::string h(line);
        while (!h.empty() && (h.back() == '\n' || h.back() == '\r')) h.pop_back();
        ok = h == tune_header(device_name);
    }
    std::lock_guard<std::mutex> lk(tune_mtx);
    unsigned b = 0;
    int best = -1;
    while (ok && std::fscanf(f, "%u %d", &b, &best) == 2)
        if (best >= 0 && best < kNumShapes) {
            TuneEntry& t = tune[b];
            t.ms.assign(kNumShapes, INFINITY);
            t.best = best;
            t.reports = kNumShapes * kTuneReps;
        }
    std::fclose(f);
}

void Ctx::tune_save()
{
    if (tune_path.empty()) return;
    std::lock_guard<std::mutex> lk(tune_mtx);
    const std::string tmp = tune_path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "%s\n", tune_header(device_name).c_str());
    for (const auto& kv : tune)
        if (kv.second.best >= 0) std::fprintf(f, "%u %d\n", kv.first, kv.second.best);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), tune_path.c_str());
}

Ctx::~Ctx()
{
    tune_save();
    {
        std::lock_guard<std::mutex> lk(qmtx);
        stopping = true;
    }
    qcv.notify_all();
    for (auto& w : workers)
        if (w.joinable()) w.join();
    for (auto& s : slots) {
        if (!s) continue;
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        for (auto& e : s->ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& g : s->graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (s->stream) (void)hipStreamDestroy(s->stream);
    }
    if (tbl_stream) (void)hipStreamDestroy(tbl_stream);
}

mcd_status Ctx::start(int nslots)
{
    if (hipStreamCreateWithFlags(&tbl_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        err = "stream creation failed";
        return MCD_E_HIP;
    }
    for (int i = 0; i < nslots; ++i) {
        auto s = std::make_unique<Slot>();
        s->cand_cap = cand_cap0;
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            err = "stream creation failed";
            return MCD_E_HIP;
        }
        for (auto& e : s->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                err = "event creation failed";
                return MCD_E_HIP;
            }
        slots.push_back(std::move(s));
    }
    for (int i = 0; i < nslots; ++i) workers.emplace_back(&Ctx::worker, this, i);
    return MCD_OK;
}

}  // namespace mcd

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

int32_t mcd_abi_version(void) { return MCD_ABI_VERSION; }

mcd_status mcd_create(const mcd_config* cfg, void* stream, mcd_ctx** out)
{
    if (!out) { g_create_error = "mcd_create: out is NULL"; return MCD_E_INVALID; }
    *out = nullptr;
    mcd_config d{};
    if (cfg) d = *cfg;
    if ((d.flags & ~(MCD_CFG_NO_GRAPHS | MCD_CFG_NO_TUNE)) != 0) {
        g_create_error = "mcd_create: unknown config flags";
        return MCD_E_INVALID;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        g_create_error = "mcd_create: no HIP device";
        return MCD_E_HIP;
    }
    Ctx* c = new (std::nothrow) Ctx();
    if (!c) { g_create_error = "mcd_create: host allocation failed"; return MCD_E_OOM; }
    c->mem_budget = d.mem_budget > 0 ? d.mem_budget : (int64_t)8 << 30;
    c->n_streams = d.streams > 0 ? std::min(d.streams, 8) : 2;
    c->margin_c = d.margin_c > 0 ? d.margin_c : 256.0;
    c->cand_cap0 = d.contact_cap > 0 ? d.contact_cap : (1 << 20);
    c->device = dev;
    c->num_cu = prop.multiProcessorCount;
    c->user_stream = (hipStream_t)stream;
    c->grid32 = c->num_cu * 16;
    c->grid64 = c->num_cu * 8;
    c->use_graphs = (d.flags & MCD_CFG_NO_GRAPHS) == 0;
    c->use_tune = (d.flags & MCD_CFG_NO_TUNE) == 0;
    c->device_name = std::string(prop.gcnArchName) + "-" + std::to_string(prop.multiProcessorCount) + "cu";
    for (char& ch : c->device_name)
        if (ch == ' ') ch = '_';
    if (d.tune_cache && c->use_tune) {
        c->tune_path = d.tune_cache;
        c->tune_load();
    }
    mcd_status st = c->start(c->n_streams);
    if (st == MCD_OK) st = scratch_setup(dev, c->err);
    if (st != MCD_OK) {
        g_create_error = "mcd_create: " + c->err;
        delete c;
        return st;
    }
    *out = reinterpret_cast<mcd_ctx*>(c);
    return MCD_OK;
}

void mcd_destroy(mcd_ctx* ctx)
{
    if (!ctx) return;
    delete reinterpret_cast<Ctx*>(ctx);
}

const char* mcd_last_error(const mcd_ctx* ctx)
{
    if (!ctx) return g_create_error.c_str();
    return reinterpret_cast<const Ctx*>(ctx)->err.c_str();
}

#define CTX_GUARD                                                     \
    if (!ctx) return MCD_E_INVALID;                                   \
    Ctx* c = reinterpret_cast<Ctx*>(ctx);                             \
    std::lock_guard<std::mutex> lk(c->mtx);                           \
    try {
#define CTX_END                                                       \
    } catch (const std::bad_alloc&) {                                 \
        c->err = "host allocation failed";                            \
        return MCD_E_OOM;                                             \
    } catch (...) {                                                   \
        c->err = "internal error";                                    \
        return MCD_E_INVALID;                                         \
    }

mcd_status mcd_mesh_load(mcd_ctx* ctx, const double* xyz, int32_t nv, const int32_t* tri, int32_t nt,
                         double halo_eps, int32_t* mesh_id)
{
    CTX_GUARD
    return c->mesh_load(xyz, nv, tri, nt, halo_eps, mesh_id);
    CTX_END
}

mcd_status mcd_mesh_unload(mcd_ctx* ctx, int32_t mesh_id)
{
    CTX_GUARD
    if (mesh_id < 0 || mesh_id >= (int32_t)c->meshes.size() || !c->meshes[mesh_id].alive) {
        c->err = "mesh_unload: unknown mesh id";
        return MCD_E_NOT_FOUND;
    }
    c->wait_no_readers();
    c->meshes[mesh_id].alive = false;
    return c->upload_meshes();
    CTX_END
}

mcd_status mcd_particles_set(mcd_ctx* ctx, int32_t n, const int32_t* pid, const int32_t* mesh_id,
                             const mcd_state* s)
{
    CTX_GUARD
    return c->particles_set(n, pid, mesh_id, s);
    CTX_END
}

static mcd_status submit_pairs(Ctx* c, const int32_t* pairs, int32_t n, const mcd_qopts* o,
                               uint64_t* ticket, std::chrono::steady_clock::time_point t0)
{
    if (n < 0 || (n > 0 && !pairs) || !ticket) { c->err = "query: invalid arguments"; return MCD_E_INVALID; }
    auto q = std::make_shared<Query>();
    mcd_status st = c->check_opts(o, q->opts);
    if (st != MCD_OK) return st;
    st = c->prepare_pairs(pairs, n, *q, c->err);
    if (st != MCD_OK) return st;
    q->stats.submit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return c->enqueue(q, ticket);
}

mcd_status mcd_query_pairs(mcd_ctx* ctx, int32_t n, const int32_t* pid_pairs, const mcd_qopts* o,
                           uint64_t* ticket)
{
    const auto t0 = std::chrono::steady_clock::now();
    CTX_GUARD
    return submit_pairs(c, pid_pairs, n, o, ticket, t0);
    CTX_END
}

mcd_status mcd_query_pairs_dev(mcd_ctx* ctx, int32_t n, const int32_t* d_pairs, const mcd_qopts* o,
                               void* stream, uint64_t* ticket)
{
    const auto t0 = std::chrono::steady_clock::now();
    CTX_GUARD
    if (n < 0 || (n > 0 && !d_pairs) || !ticket) { c->err = "query_pairs_dev: invalid arguments"; return MCD_E_INVALID; }
    auto q = std::make_shared<Query>();
    mcd_status st = c->check_opts(o, q->opts);
    if (st != MCD_OK) return st;
    q->dev = true;
    q->d_list = d_pairs;
    q->n_dev = n;
    // the list is read once the work queued on the caller's stream is done
    if (n > 0) {
        hipStream_t cs = stream ? (hipStream_t)stream : c->user_stream;
        if (!c->hip_ok(hipEventCreateWithFlags(&q->ready, hipEventDisableTiming), "event") ||
            !c->hip_ok(hipEventRecord(q->ready, cs), "event"))
            return MCD_E_HIP;
    }
    // the tile pairs are counted on the device; the working-set estimate
    // assumes 64 per pair until a run of the query has counted them
    q->tile_pairs_total = (int64_t)n * 64;
    q->mem_estimate = q->tile_pairs_total * 48 +
                      (int64_t)n * (1024 + (q->opts.dt > 0.0 ? (int64_t)(q->opts.samples + 1) * 144 : 0));
    q->stats.submit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return c->enqueue(q, ticket);
    CTX_END
}

mcd_status mcd_query_cluster(mcd_ctx* ctx, int32_t n, const int32_t* pid, const mcd_state* states,
                             const mcd_qopts* o, uint64_t* ticket)
{
    const auto t0 = std::chrono::steady_clock::now();
    CTX_GUARD
    if (!ticket || n < 0 || (n > 0 && !pid)) { c->err = "query_cluster: invalid arguments"; return MCD_E_INVALID; }
    mcd_qopts opts;
    mcd_status st = c->check_opts(o, opts);
    if (st != MCD_OK) return st;
    bool on_device = true;
    for (int i = 0; i < n; ++i)
        if (pid[i] < 0 || pid[i] >= DEV_PID_LIMIT) on_device = false;
    if (!on_device) {
        // ids beyond the device table: pairs found on the host
        std::vector<int32_t> pairs;
        st = c->cluster_pairs(n, pid, states, opts, pairs);
        if (st != MCD_OK) return st;
        return submit_pairs(c, pairs.data(), (int32_t)(pairs.size() / 2), &opts, ticket, t0);
    }
    // members checked on the host (known ids, each once); new states first
    {
        std::vector<int32_t> ids(pid, pid + n);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end()) {
            c->err = "query_cluster: particle listed twice";
            return MCD_E_INVALID;
        }
    }
    std::vector<int32_t> mids;
    if (states) mids.resize(n);
    for (int i = 0; i < n; ++i) {
        auto it = c->particles.find(pid[i]);
        if (it == c->particles.end()) {
            c->err = "query_cluster: unknown particle " + std::to_string(pid[i]);
            return MCD_E_NOT_FOUND;
        }
        if (!c->meshes[it->second.mesh].alive) {
            c->err = "query_cluster: particle " + std::to_string(pid[i]) + " uses an unloaded mesh";
            return MCD_E_NOT_FOUND;
        }
        if (states) mids[i] = it->second.mesh;
    }
    if (states && (st = c->particles_set(n, pid, mids.data(), states)) != MCD_OK) return st;
    // the candidate pairs are found on the device (section 3, checks 1 and
    // 2) and read in place by the contact query
    auto q = std::make_shared<Query>();
    q->opts = opts;
    q->dev = q->cluster = true;
    q->members.assign(pid, pid + n);
    q->seg_off = {0, n};
    const int64_t all_pairs = (int64_t)n * (n - 1) / 2;
    q->n_dev = (int32_t)std::min<int64_t>(all_pairs, 8 * (int64_t)n + 16);
    q->tile_pairs_total = (int64_t)q->n_dev * 16;
    q->mem_estimate = q->tile_pairs_total * 48 +
                      (int64_t)q->n_dev * (1024 + (opts.dt > 0.0 ? (int64_t)(opts.samples + 1) * 144 : 0));
    q->stats.submit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return c->enqueue(q, ticket);
    CTX_END
}

mcd_status mcd_impulses(mcd_ctx* ctx, int32_t n, const int32_t* pid_pairs, const mcd_contact* contacts,
                        const mcd_impulse_opts* o, double* impulse, int32_t* n_particles, int32_t* pids_out,
                        double* vel_out, int32_t* sweeps)
{
    CTX_GUARD
    return c->impulses(n, pid_pairs, contacts, o, impulse, n_particles, pids_out, vel_out, sweeps);
    CTX_END
}

mcd_status mcd_broad_phase(mcd_ctx* ctx, int32_t n, const int32_t* pid, double dt, int32_t* cluster,
                           int32_t* n_clusters, int32_t* pairs_out, int64_t cap_pairs, int64_t* n_pairs)
{
    CTX_GUARD
    c->wait_no_readers();
    return c->broad_phase(n, pid, dt, cluster, n_clusters, pairs_out, cap_pairs, n_pairs);
    CTX_END
}

// Look up a ticket under the context lock, then wait on it without the lock.
static std::shared_ptr<Query> lookup(Ctx* c, uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(c->mtx);
    return c->find(ticket);
}

static mcd_status wait_done(Ctx* c, Query& q, int64_t timeout_ns)
{
    std::unique_lock<std::mutex> lk(q.m);
    if (timeout_ns < 0) {
        q.cv.wait(lk, [&] { return q.done; });
    } else if (!q.cv.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return q.done; })) {
        std::lock_guard<std::mutex> g(c->mtx);
        c->err = "wait: timed out";
        return MCD_E_TIMEOUT;
    }
    if (q.status != MCD_OK) {
        std::lock_guard<std::mutex> g(c->mtx);
        c->err = q.err;
    }
    return q.status;
}

mcd_status mcd_poll(mcd_ctx* ctx, uint64_t ticket, int32_t* done)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    std::lock_guard<std::mutex> lk(q->m);
    if (done) *done = q->done ? 1 : 0;
    return MCD_OK;
}

mcd_status mcd_wait(mcd_ctx* ctx, uint64_t ticket, int64_t timeout_ns)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    return wait_done(c, *q, timeout_ns);
}

mcd_status mcd_result_sizes(mcd_ctx* ctx, uint64_t ticket, int32_t* n_pairs, int64_t* n_contacts)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    mcd_status st = wait_done(c, *q, -1);
    if (st != MCD_OK) return st;
    if (n_pairs) *n_pairs = (int32_t)(q->pairs.size() / 2);
    if (n_contacts) *n_contacts = q->ncon;
    return MCD_OK;
}

// Contact records copied out in a few host threads when there are many: a
// caller's freshly allocated array faults its pages in on first touch, and
// the faults of different pages are served in parallel. Pair indices are
// re-based on the way (base 0: a plain copy).
static void copy_contacts(mcd_contact* dst, const mcd_contact* src, size_t n, int32_t base)
{
    auto part = [&](size_t lo, size_t hi) {
        if (base == 0) {
            std::memcpy(dst + lo, src + lo, (hi - lo) * sizeof(mcd_contact));
            return;
        }
        for (size_t i = lo; i < hi; ++i) {
            dst[i] = src[i];
            dst[i].pair -= base;
        }
    };
    constexpr size_t kPerThread = (size_t)4 << 20;   // bytes below which one thread copies
    const size_t bytes = n * sizeof(mcd_contact);
    const size_t nt = bytes < 2 * kPerThread
                          ? 1
                          : std::min<size_t>({(size_t)8, (size_t)host_threads(), bytes / kPerThread});
    if (nt <= 1) {
        part(0, n);
        return;
    }
    // parts whose thread cannot be started are copied here
    std::vector<std::thread> ts;
    ts.reserve(nt - 1);
    size_t started = 1;
    try {
        for (; started < nt; ++started) ts.emplace_back(part, n * started / nt, n * (started + 1) / nt);
    } catch (const std::system_error&) {
    }
    for (size_t t = started; t < nt; ++t) part(n * t / nt, n * (t + 1) / nt);
    part(0, n / nt);
    for (auto& t : ts) t.join();
}

mcd_status mcd_fetch(mcd_ctx* ctx, uint64_t ticket, mcd_pair_result* pr, int32_t cap_pairs,
                     mcd_contact* contacts, int64_t cap_contacts, int32_t* pairs_out)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    mcd_status st = wait_done(c, *q, -1);
    if (st != MCD_OK) return st;
    const size_t np = q->pairs.size() / 2, nc = (size_t)q->ncon;
    if ((pr && (size_t)cap_pairs < np) || (pairs_out && (size_t)cap_pairs < np) ||
        (contacts && (size_t)cap_contacts < nc)) {
        std::lock_guard<std::mutex> g(c->mtx);
        c->err = "fetch: capacity too small";
        return MCD_E_INVALID;
    }
    if (contacts && q->dout) {
        std::lock_guard<std::mutex> g(c->mtx);
        c->err = "fetch: the contact records are in device memory (MCD_Q_DEVICE_OUT): use mcd_fetch_dev";
        return MCD_E_INVALID;
    }
    if (pr && np) std::memcpy(pr, q->result.data(), np * sizeof(mcd_pair_result));
    if (contacts && nc) {
        std::lock_guard<std::mutex> g(q->m);
        copy_contacts(contacts, q->cdata(), nc, q->rebased ? 0 : q->pair_base);
    }
    if (pairs_out && np) std::memcpy(pairs_out, q->pairs.data(), 2 * np * sizeof(int32_t));
    return MCD_OK;
}

mcd_status mcd_result_view(mcd_ctx* ctx, uint64_t ticket, const mcd_pair_result** pr,
                           const mcd_contact** contacts, const int32_t** pairs)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    mcd_status st = wait_done(c, *q, -1);
    if (st != MCD_OK) return st;
    if (pr) *pr = q->result.data();
    if (contacts && !q->dout && q->ncon > 0) {
        std::lock_guard<std::mutex> g(q->m);
        mcd_contact* cd = q->cdata();
        if (!q->rebased) {   // this query's own range of the batch's records
            for (int64_t i = 0; i < q->ncon; ++i) cd[i].pair -= q->pair_base;
            q->rebased = true;
        }
        *contacts = cd;
    } else if (contacts) {
        *contacts = nullptr;
    }
    if (pairs) *pairs = q->pairs.data();
    return MCD_OK;
}

mcd_status mcd_fetch_dev(mcd_ctx* ctx, uint64_t ticket, mcd_pair_result* d_pr, int32_t cap_pairs,
                         mcd_contact* d_contacts, int64_t cap_contacts, void* stream)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    mcd_status st = wait_done(c, *q, -1);
    if (st != MCD_OK) return st;
    const size_t np = q->pairs.size() / 2, nc = (size_t)q->ncon;
    const char* why = nullptr;
    if (!q->dout) why = "fetch_dev: the query was not submitted with MCD_Q_DEVICE_OUT";
    else if ((d_pr && (size_t)cap_pairs < np) || (d_contacts && (size_t)cap_contacts < nc))
        why = "fetch_dev: capacity too small";
    if (why) {
        std::lock_guard<std::mutex> g(c->mtx);
        c->err = why;
        return MCD_E_INVALID;
    }
    hipStream_t cs = stream ? (hipStream_t)stream : c->user_stream;
    std::lock_guard<std::mutex> g(q->m);
    if (!c->hip_ok(hipSetDevice(c->device), "fetch_dev") ||
        !c->hip_ok(hipStreamWaitEvent(cs, q->dev_done, 0), "fetch_dev") ||
        (d_pr && np && !c->hip_ok(hipMemcpyAsync(d_pr, q->dout->p, sizeof(mcd_pair_result) * np,
                                                 hipMemcpyDeviceToDevice, cs), "fetch_dev")) ||
        (d_contacts && nc && !c->hip_ok(hipMemcpyAsync(d_contacts, (const char*)q->dout->p + q->dout_con,
                                                       sizeof(mcd_contact) * nc, hipMemcpyDeviceToDevice, cs),
                                        "fetch_dev")) ||
        (!q->fetched && !c->hip_ok(hipEventCreateWithFlags(&q->fetched, hipEventDisableTiming), "fetch_dev")) ||
        !c->hip_ok(hipEventRecord(q->fetched, cs), "fetch_dev"))
        return MCD_E_HIP;
    return MCD_OK;
}

mcd_status mcd_cluster_time(mcd_ctx* ctx, uint64_t ticket, double* t_new)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    if (!t_new) return MCD_E_INVALID;
    mcd_status st = wait_done(c, *q, -1);
    if (st != MCD_OK) return st;
    double t = q->opts.dt;
    for (const auto& r : q->result)
        if (r.status == MCD_COLLIDES && r.toi < t) t = r.toi;
    *t_new = t;
    return MCD_OK;
}

mcd_status mcd_query_stats(mcd_ctx* ctx, uint64_t ticket, mcd_stats* out)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    auto q = lookup(c, ticket);
    if (!q) return MCD_E_NOT_FOUND;
    if (!out) return MCD_E_INVALID;
    mcd_status st = wait_done(c, *q, -1);
    if (st != MCD_OK) return st;
    *out = q->stats;
    return MCD_OK;
}

mcd_status mcd_release(mcd_ctx* ctx, uint64_t ticket)
{
    CTX_GUARD
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) { c->err = "release: unknown ticket"; return MCD_E_NOT_FOUND; }
    c->tickets.erase(it);
    return MCD_OK;
    CTX_END
}

}  // extern "C"

// ======================================================================
// Allocation-free static contact query
// ======================================================================
// Every device buffer of the query beyond its inputs and outputs comes from
// one file-scope device array of fixed size. Its address is taken once per
// device at context creation (the host-side name is not a device address).
// Calls in one process are serialised; calls that overlapped on one GPU
// would race on the array.
namespace mcd {
namespace noalloc {

constexpr int64_t kPairs = 1 << 14;            // particle pairs per call
constexpr int64_t kTilePairs = 1 << 24;        // tile pairs spanned by the pairs of a call
constexpr int64_t kItems = 1 << 20;            // tile pairs kept by the cull
constexpr int64_t kNear = 1 << 22;             // near triangle pairs
constexpr int64_t kCands = 1 << 19;            // candidates of the FP64 re-decision
constexpr int64_t kWords = kTilePairs / 64 + kPairs + 1;

constexpr int64_t up(int64_t x) { return (x + 255) & ~(int64_t)255; }
// byte offsets of the regions
constexpr int64_t oCounters = 0;
constexpr int64_t oNlist = up(oCounters + 4 * NCOUNTERS);
constexpr int64_t oStats = up(oNlist + 256);
constexpr int64_t oSrc = up(oStats + 8 * (int64_t)STAT_ROWS * STAT_WAVES);
constexpr int64_t oPairs = up(oSrc + (int64_t)PAIR_HDR + (int64_t)sizeof(PairSrc) * kPairs);
constexpr int64_t oGather = up(oPairs + (int64_t)PAIR_HDR + (int64_t)sizeof(PairDev) * kPairs);
constexpr int64_t oScan = up(oGather + 16 * kPairs);
constexpr int64_t oUb = up(oScan + (int64_t)(2 * ((kPairs + 1) & ~1)) * 4 + kPairs * 8 + 16);
constexpr int64_t oD2 = up(oUb + 4 * kPairs);
constexpr int64_t oTie = up(oD2 + 8 * kPairs);
constexpr int64_t oCnt = up(oTie + 8 * kPairs);
constexpr int64_t oOff = up(oCnt + 4 * kPairs);
constexpr int64_t oLarge = up(oOff + 4 * (kPairs + 1));
constexpr int64_t oMask = up(oLarge + 4 * kPairs);
constexpr int64_t oItems = up(oMask + 8 * kWords);
constexpr int64_t oNear = up(oItems + (int64_t)sizeof(NearItem) * kItems);
constexpr int64_t oCands = up(oNear + (int64_t)sizeof(NearRec) * kNear);
constexpr int64_t oOuts = up(oCands + (int64_t)sizeof(Cand) * kCands);
constexpr int64_t oCkey = up(oOuts + (int64_t)sizeof(CandOut) * kCands);
constexpr int64_t oCd2 = up(oCkey + 8 * kCands);
constexpr int64_t oSeg = up(oCd2 + 8 * kCands);
constexpr int64_t kBytes = up(oSeg + 8 * kCands);
static_assert(kBytes <= ((int64_t)160 << 20), "scratch layout exceeds its stated size");
static_assert(sizeof(PairOut) == sizeof(mcd_pair_result), "pair results are written in place");

}  // namespace noalloc
}  // namespace mcd

static __device__ __align__(256) unsigned char scratch[mcd::noalloc::kBytes];

namespace mcd {

static std::mutex g_scratch_mtx;          // the address table and the calls
static std::map<int, void*> g_scratch;    // device -> address of its scratch array

// Once per device, with that device current (context creation).
static mcd_status scratch_setup(int device, std::string& err)
{
    std::lock_guard<std::mutex> lk(g_scratch_mtx);
    if (g_scratch.count(device)) return MCD_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        err = std::string("scratch address: ") + hipGetErrorString(e);
        return MCD_E_HIP;
    }
    g_scratch[device] = ptr;
    return MCD_OK;
}

mcd_status Ctx::query_noalloc(int32_t n, const int32_t* d_pairs, hipStream_t st, mcd_pair_result* d_results,
                              mcd_contact* d_contacts, int64_t cap_contacts, int64_t* n_contacts)
{
    using namespace noalloc;
    if (n < 0 || n > kPairs || (n > 0 && (!d_pairs || !d_results)) || cap_contacts < 0 ||
        (cap_contacts > 0 && !d_contacts)) {
        err = "query_pairs_noalloc: invalid arguments (at most " + std::to_string(kPairs) + " pairs)";
        return MCD_E_INVALID;
    }
    if (n_contacts) *n_contacts = 0;
    if (n == 0) return MCD_OK;
    std::lock_guard<std::mutex> lk(g_scratch_mtx);
    auto it = g_scratch.find(device);
    if (it == g_scratch.end()) { err = "query_pairs_noalloc: no scratch address for this device"; return MCD_E_HIP; }
    char* base = (char*)it->second;
    int32_t* c = (int32_t*)(base + oCounters);
    unsigned long long* c64 = (unsigned long long*)c;
    int32_t* nlist = (int32_t*)(base + oNlist);
    unsigned long long* sl = (unsigned long long*)(base + oStats);
    int32_t* hsrc = (int32_t*)(base + oSrc);
    PairSrc* src = (PairSrc*)(base + oSrc + PAIR_HDR);
    int32_t* hpairs = (int32_t*)(base + oPairs);
    PairDev* dp = (PairDev*)(base + oPairs + PAIR_HDR);
    NearItem* items = (NearItem*)(base + oItems);
    NearRec* nr = (NearRec*)(base + oNear);
    Cand* cands = (Cand*)(base + oCands);
    CandOut* outs = (CandOut*)(base + oOuts);
    const int32_t pc = (int32_t)kPairs;
    Launch L{st, num_cu};
    TriStore S = store();
    PrepOpts popt{};
    popt.dt = 0.0;
    popt.tol_rel = 1e-6;
    popt.margin_c = margin_c;
    popt.samples = 64;
    popt.flags = (int32_t)(MCD_Q_MIXED | MCD_Q_CLOSEST | MCD_Q_CONTACTS);
    const int gnear = num_cu * kShapes[0].near_wpc, geval = num_cu * kShapes[0].eval_wpc;
    const int grec = recheck_grid(kCands);
    const StatPlan plan{7, {2 * gnear, geval, 0, grec, 2 * gnear, grec, grec}, {7, 5, 6, 8, 9, 12, 13}};
    // the chain of the device-list query, launched on the caller's stream
    bool ok = hip_ok(launch_fill_u32(L, (uint32_t*)nlist, 1, (uint32_t)n), "no-alloc query") &&
              hip_ok(launch_init_static(L, (uint32_t*)c, NCOUNTERS, (uint32_t*)(base + oUb), (uint64_t*)(base + oD2),
                                        (uint64_t*)(base + oTie), (int32_t*)(base + oCnt), pc), "no-alloc query") &&
              hip_ok(launch_pair_gather(L, nlist, d_pairs, pc, (const PartDev*)dpart.p, dpart_cap,
                                        (const MeshDev*)dmesh.p, (int32_t)meshes.size(), 0.0, 0, 1, kTilePairs, kWords,
                                        hsrc, src, (int64_t*)(base + oGather), c, 29, 11, 15, 16), "no-alloc query") &&
              hip_ok(launch_pair_prep(L, hsrc, src, pc, popt, hpairs, dp), "no-alloc query") &&
              hip_ok(launch_cull(L, dp, hpairs, pc, S, 0, nullptr, items, c + 0, kItems, c64 + 4,
                                 (int32_t*)(base + oScan), (uint64_t*)(base + oMask)), "no-alloc query") &&
              hip_ok(launch_near(L, dp, S, items, c + 0, kItems, c + 64, nr, c + 6, kNear, sl, sl + 4 * STAT_WAVES,
                                 gnear), "no-alloc query") &&
              hip_ok(launch_eval(L, false, dp, S, nr, c + 6, kNear, cands, c + 1, kCands, sl + STAT_WAVES, geval),
                     "no-alloc query") &&
              hip_ok(launch_recheck(L, dp, S, cands, c + 1, kCands, outs, (uint64_t*)(base + oCkey),
                                    (uint64_t*)(base + oCd2), (uint64_t*)(base + oD2), (int32_t*)(base + oCnt),
                                    sl + 3 * STAT_WAVES, sl + 5 * STAT_WAVES, sl + 6 * STAT_WAVES,
                                    (uint32_t*)(c + 34)), "no-alloc query") &&
              hip_ok(launch_pair_scan(L, hpairs, (int32_t*)(base + oCnt), (int32_t*)(base + oOff), c + 20,
                                      (int32_t*)(base + oLarge)), "no-alloc query") &&
              hip_ok(launch_tie_out(L, (uint64_t*)(base + oCkey), (uint64_t*)(base + oCd2), c + 1, kCands,
                                    (uint64_t*)(base + oD2), (uint64_t*)(base + oTie)), "no-alloc query") &&
              hip_ok(launch_pair_final(L, dp, hpairs, pc, S, (uint64_t*)(base + oD2), (uint64_t*)(base + oTie), 0,
                                       (PairOut*)d_results), "no-alloc query") &&
              hip_ok(launch_stat_reduce(L, (const uint64_t*)sl, plan, c64), "no-alloc query");
    int32_t hc[64];
    ok = ok && hip_ok(hipMemcpyAsync(hc, c, sizeof hc, hipMemcpyDeviceToHost, st), "no-alloc query") &&
         hip_ok(hipStreamSynchronize(st), "no-alloc query");
    if (!ok) return MCD_E_HIP;
    const int64_t* hc64 = (const int64_t*)hc;
    const int32_t gerr = hc[29];
    if (gerr & (GATHER_BAD_ID | GATHER_DEAD_MESH)) {
        err = "query_pairs_noalloc: unknown particle id (or an id >= 2^24) or an unloaded mesh in the pair list";
        return MCD_E_NOT_FOUND;
    }
    if (gerr & GATHER_SAME) { err = "query_pairs_noalloc: a pair repeats a particle"; return MCD_E_INVALID; }
    if ((gerr & GATHER_OVERFLOW) || hc[0] > kItems || hc[6] > kNear || hc[1] > kCands) {
        err = "query_pairs_noalloc: the query exceeds the fixed scratch (limits: " + std::to_string(kTilePairs) +
              " tile pairs spanned, " + std::to_string(kItems) + " kept, " + std::to_string(kNear) +
              " near triangle pairs, " + std::to_string(kCands) + " candidates)";
        return MCD_E_INVALID;
    }
    const int64_t nout = hc64[8];
    if (n_contacts) *n_contacts = nout;
    if (nout > 0) {
        const int32_t maxseg = hc[20];
        if (maxseg > SEG_CAP) {
            err = "query_pairs_noalloc: a pair has more than " + std::to_string(SEG_CAP) + " contacts";
            return MCD_E_INVALID;
        }
        if (nout > cap_contacts) { err = "query_pairs_noalloc: contact capacity too small"; return MCD_E_INVALID; }
        int p2 = 1;
        while (p2 < maxseg) p2 <<= 1;
        if (!hip_ok(sort_contacts_by_pair(L, outs, (uint64_t*)(base + oCkey), hc[1], n, (int32_t*)(base + oOff),
                                          (int32_t*)(base + oCnt), (const int32_t*)(base + oLarge),
                                          std::min(hc[21], n), (uint64_t*)(base + oSeg), p2, d_contacts),
                    "no-alloc query") ||
            !hip_ok(hipStreamSynchronize(st), "no-alloc query"))
            return MCD_E_HIP;
    }
    return MCD_OK;
}

}  // namespace mcd

extern "C" mcd_status mcd_query_pairs_noalloc(mcd_ctx* ctx, int32_t n, const int32_t* d_pairs, void* stream,
                                              mcd_pair_result* d_results, mcd_contact* d_contacts,
                                              int64_t cap_contacts, int64_t* n_contacts)
{
    if (!ctx) return MCD_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mtx);
    try {
        return c->query_noalloc(n, d_pairs, stream ? (hipStream_t)stream : c->user_stream, d_results, d_contacts,
                                cap_contacts, n_contacts);
    } catch (...) {
        c->err = "internal error";
        return MCD_E_INVALID;
    }
}
