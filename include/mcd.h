/*
 * mcd.h - narrow-phase contact detection between rigid particles represented
 * by triangulated meshes, on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Noble & Weinzierl, "Parallel local time stepping for
 * rigid bodies represented by triangulated meshes":
 *  - a particle is a rigid triangle mesh with a halo of width eps (section 2,
 *    "Physical model"); two particles touch when their halos overlap, i.e.
 *    when some triangle pair is at distance d <= eps_a + eps_b (section 5,
 *    "Geometric model" and the contact-point definition);
 *  - a contact carries a position (midpoint of the closest points), a time
 *    stamp, the shortest distance vector and the two triangles (contact-point
 *    definition, section 5);
 *  - motion within a step is linear in position and spherical-linear in the
 *    rotation quaternion, i.e. constant v and world-frame angular velocity w
 *    (section 2, "Physical model");
 *  - the collision time stamp of a pair is the first time in [0, dt] at which
 *    its halos overlap; pairs in contact at the start or moving apart do not
 *    constrain the step (section 5, case distinctions); a cluster's new time
 *    is the minimum over its colliding pairs (section 5, update of t_new).
 *
 * Conventions for every call:
 *  - Return value: MCD_OK or a negative mcd_status. No call throws or aborts
 *    across this boundary. On error, mcd_last_error(ctx) describes it.
 *  - Host pointers are read during the call only and stay owned by the
 *    caller. Device pointers (the *_dev variants) must stay valid until the
 *    ticket that used them completes.
 *  - Triangle ids in results are the caller's ids: the index of the face in
 *    the array given to mcd_mesh_load.
 *  - Calls on one context are serialised by an internal mutex; a context is
 *    bound to the device that was current at mcd_create.
 */
#ifndef MCD_H
#define MCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCD_ABI_VERSION 2

typedef enum {
    MCD_OK = 0,
    MCD_E_INVALID = -1,   /* bad argument or input geometry */
    MCD_E_OOM = -2,       /* device or host allocation failed; the context stays usable */
    MCD_E_NOT_FOUND = -3, /* unknown mesh id, particle id or ticket */
    MCD_E_BUSY = -4,      /* admission refused: the query does not fit the memory budget now */
    MCD_E_TIMEOUT = -5,   /* mcd_wait ran out of time; the ticket is still valid */
    MCD_E_HIP = -6        /* a HIP runtime call failed */
} mcd_status;

typedef struct mcd_ctx mcd_ctx;

/* Context configuration. Zero-initialised fields take the defaults shown. */
typedef struct {
    int64_t mem_budget;     /* bytes of device memory for query working sets; 0: 8 GiB. Admission
                               counts each query's estimated working set (tile pairs and pair
                               records) against it; the per-stream workspaces, which keep the size
                               of the largest query they ran, are not counted */
    int32_t streams;        /* streams for concurrently executing batches (serving); 0: 2 */
    double margin_c;        /* FP32 filter margin in units of 2^-23 * scale; 0: 256 */
    int32_t contact_cap;    /* initial capacity of candidate/contact buffers; 0: 1<<20 */
    int32_t flags;          /* MCD_CFG_* bits; 0: defaults */
    const char* tune_cache; /* file of the autotuner's choices, read at creation and written at
                               destruction (NULL: none). Entries of another device model or
                               another set of launch shapes are ignored. */
} mcd_config;

/* Context flags. */
enum {
    MCD_CFG_NO_GRAPHS = 1 << 0,   /* launch kernel chains one by one instead of replaying captured
                                     HIP graphs */
    MCD_CFG_NO_TUNE = 1 << 1      /* fixed launch shapes: no autotuning */
};

/* Rigid state of a particle at the start of the step. */
typedef struct {
    double x[3];   /* centre of rotation, world frame */
    double q[4];   /* rotation quaternion (w, x, y, z), body to world; normalised on ingest */
    double v[3];   /* linear velocity */
    double w[3];   /* angular velocity, world frame (rad per time unit) */
} mcd_state;

/* Query flags. */
enum {
    MCD_Q_FP64 = 1u << 0,     /* every triangle pair in FP64 (plain FP64 kernel) */
    MCD_Q_MIXED = 1u << 1,    /* FP32 filter, FP64 re-decision near the threshold (default) */
    MCD_Q_DENSE = 1u << 2,    /* evaluate all triangle pairs: no tile culling, exact minimum for
                                 every pair even beyond the halo */
    MCD_Q_TIMING = 1u << 3,   /* launch the kernels one by one with an event between each, so that
                                 mcd_query_stats reports per-kernel device times; otherwise a static
                                 query replays one captured HIP graph of its kernel chain */
    MCD_Q_CLOSEST = 1u << 4,  /* report each pair's minimum distance, its closest points and its
                                 triangle pair (section 5, shortest distance vector of the
                                 contact-point definition) */
    MCD_Q_CONTACTS = 1u << 5, /* report the contact records (section 5, contact-point
                                 definition). Neither CLOSEST nor CONTACTS set means both. Without
                                 CONTACTS no record is sorted or copied back (mcd_result_sizes
                                 reports 0 contacts); without CLOSEST a pair result carries its
                                 contact flag, status and time stamp, with dmin = +inf, tri_a =
                                 tri_b = -1 and zero points */
    MCD_Q_VALIDATE = 1u << 6, /* diagnostic for MIXED queries: every triangle pair the FP32 filter
                                 evaluates is re-evaluated in FP64, and mcd_stats.margin_ratio
                                 reports the largest |d32 - d64| over the FP32 margin. The
                                 results are those of the same query without this flag */
    MCD_Q_FUSE = 1u << 8,     /* contact fusion (section 5, after the contact-point definition:
                                 contact points close in space become one, centred within
                                 parallel triangles): per pair, in (tri_a, tri_b) order, the first
                                 record not yet fused seeds a group and the later ones whose
                                 contact point lies within eps_a + eps_b of the seed's join it; a
                                 group is returned as one record with the seed's triangles, the
                                 mean contact point and the distance vector of its member nearest
                                 to contact; `merged` counts its members */
    MCD_Q_DEVICE_OUT = 1u << 9, /* static queries: the pair results and the sorted contact records
                                 stay in device memory held by the ticket (no copy to the host);
                                 mcd_fetch_dev copies them into caller device memory. mcd_fetch
                                 still returns the pair results and the pair ids, but not the
                                 contact records. Such queries are not batched with others */
    MCD_Q_NARROW = 1u << 7    /* time queries: the paper's own estimate instead of the exact first
                                 contact (section 5, "Collision time detection", narrowing):
                                 rotation neglected; per round, vertices against triangles at
                                 the start and end of the span and where their paths cross the
                                 triangle's plane, edge pairs at the start, middle and end; the
                                 span narrows to the earliest contact until nothing earlier is
                                 found. FP64. Contacts are reported at that time with the same
                                 translation-only motion; mcd_stats.candidates = rounds run */
};

typedef struct {
    double dt;          /* step length; 0 = static query at the start of the step */
    uint32_t flags;     /* MCD_Q_* ; 0 means MIXED */
    int32_t samples;    /* time samples S per step for time stamps, 1..128; 0: 64 */
    double tol_rel;     /* time stamp tolerance relative to dt; 0: 1e-6 (>= 1e-7) */
} mcd_qopts;

/* Per particle-pair result. Status values. */
enum { MCD_NONE = 0, MCD_AT_START = 1, MCD_COLLIDES = 2 };

typedef struct {
    double dmin;       /* minimum triangle distance (at t = toi for time queries); +inf when not
                          reported (no contact and not DENSE) */
    double pa[3];      /* closest point on A (world frame, at toi) */
    double pb[3];      /* closest point on B */
    double toi;        /* time stamp in [0, dt] (0 for static queries); +inf if NONE */
    int32_t tri_a;     /* caller's triangle id attaining dmin (lowest (tri_a, tri_b) on ties), -1 */
    int32_t tri_b;
    int32_t contact;   /* 1 if dmin <= eps_a + eps_b */
    int32_t status;    /* MCD_NONE / MCD_AT_START / MCD_COLLIDES (time queries); static: contact */
} mcd_pair_result;

/* Contact record (section 5, contact-point definition: position, time stamp,
 * shortest distance vector and the two triangles). */
typedef struct {
    int32_t pair;      /* index of the pair in the query (cluster queries: see mcd_fetch) */
    int32_t tri_a;     /* caller's triangle ids */
    int32_t tri_b;
    int32_t merged;    /* MCD_Q_FUSE: the contact records fused into this one; 0 otherwise */
    double d;          /* triangle distance, <= eps_a + eps_b */
    double pa[3];      /* closest points, world frame; contact point x = (pa+pb)/2, */
    double pb[3];      /* normal n = (pb-pa)/2 (shortest distance vector, half length) */
    double t;          /* time of the contact within the step: 0 for static queries, the pair's
                          time stamp for time queries */
} mcd_contact;

/* Counters of the last completed query of a ticket (diagnostics). */
typedef struct {
    int64_t tile_pairs_total;     /* tile pairs spanned by the query's particle pairs */
    int64_t tile_pairs_kept;      /* after the tile cull */
    int64_t tri_pairs_covered;    /* all triangle pairs of the query's particle pairs */
    int64_t tri_pairs_evaluated;  /* full triangle-pair distance evaluations by the main kernel */
    int64_t fp64_rechecks;        /* triangle pairs re-decided in FP64 */
    int64_t refine_items;         /* work items re-run in FP64 for exact minima */
    int64_t candidates;           /* time queries: triangle pairs that entered the FP64 end-game */
    int64_t fp64_evals;           /* time queries: FP64 distance evaluations */
    int64_t grazes;               /* time queries: graze leaves (no contact) */
    int64_t fp32_samples;         /* time queries: FP32 sample evaluations of the scan */
    int64_t retries;              /* buffer regrow-and-rerun rounds */
    double gpu_ms;                /* device time of the query's kernels (transfers excluded) */
    double main_ms;               /* device time of the main distance kernel (FP32 filter for
                                     MIXED, FP64 pass for FP64, sampling for time stamps) */
    double latency_ms;            /* submit to results ready on the host */
    int32_t batch_queries;        /* queries that shared the query's batch */
    int32_t batch_pairs;          /* particle pairs in that batch */
    int64_t tri_pairs_tiled;      /* triangle pairs in the tile pairs kept by the tile cull */
    int64_t sphere_tests;         /* triangle bounding-sphere tests of the near-list stage (rows,
                                     columns and packed pairs); time queries: sphere gap
                                     evaluations of the sphere walks */
    double cull_ms;               /* device time of the tile cull (time queries: space-time cull) */
    double near_ms;               /* device time of the triangle-sphere stage (time queries: the
                                     sphere walks) */
    double sort_ms;               /* device time of the contact sort */
    double endgame_ms;            /* time queries: device time of the FP64 end-game */
    double submit_ms;             /* host time inside the submitting call (cluster pairs found, pair
                                     sources staged; the pairs are prepared on the device) */
    int64_t near_pairs;           /* triangle pairs whose bounding spheres are within reach; the
                                     plane-separation test of the near-list stage leaves
                                     tri_pairs_evaluated of them */
    int64_t banded;               /* re-decided triangle pairs whose FP64 distance lies within
                                     1e-9 * delta of the threshold delta, where two correctly
                                     rounded FP64 evaluations could decide differently (expected 0) */
    int64_t validated;            /* MCD_Q_VALIDATE: FP32 evaluations compared with FP64 */
    double margin_ratio;          /* MCD_Q_VALIDATE: largest |d32 - d64| / mu, mu the FP32 margin,
                                     over the compared pairs that do not intersect and have no
                                     near-parallel edge pair; 0 otherwise */
    double margin_ratio_np;       /* the same over pairs with a near-parallel edge pair, whose FP32
                                     bound is widened by a correction c: |d32 - d64| / (mu + c) */
    int64_t cull_tests;           /* contact-set queries: bounding-sphere tests of the tile cull, at
                                     the group level (8 tiles under one sphere) and at the tile level
                                     of the group pairs kept */
    int64_t graph_captures;       /* kernel chains captured as HIP graphs so far by the context (all
                                     stream slots; each capture costs an instantiation) */
    int32_t tune_pending;         /* autotuner measurements still to run in the query's size bucket
                                     (0 once its launch shape is chosen) */
    int32_t pad;
} mcd_stats;

/* ABI version of the loaded library (MCD_ABI_VERSION). Never fails. */
int32_t mcd_abi_version(void);

/* Create a context on the current HIP device. stream: a hipStream_t to run
 * synchronous work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL
 * for a stream owned by the context. *out receives the context. */
mcd_status mcd_create(const mcd_config* cfg, void* stream, mcd_ctx** out);

/* Destroy a context: waits for its work, frees its device memory. NULL is a no-op. */
void mcd_destroy(mcd_ctx* ctx);

/* Message of the last error on this context (or of mcd_create when ctx is NULL). */
const char* mcd_last_error(const mcd_ctx* ctx);

/* Load a mesh (section 5, "Geometric model": triangle set plus halo eps).
 * xyz: nv*3 body-frame vertex coordinates about the centre of rotation;
 * tri: nt*3 vertex indices. The arrays are copied. Rejects non-finite
 * coordinates, out-of-range indices, zero-area triangles (area <= 1e-14 *
 * squared bounding-box diagonal), nt < 1, nt > 65535 and eps < 0.
 * *mesh_id receives the new id. */
mcd_status mcd_mesh_load(mcd_ctx* ctx, const double* xyz, int32_t nv, const int32_t* tri,
                         int32_t nt, double halo_eps, int32_t* mesh_id);

/* Remove a mesh. Particles still using it become invalid for queries. */
mcd_status mcd_mesh_unload(mcd_ctx* ctx, int32_t mesh_id);

/* Insert or update particles (section 2, "Physical model": a particle is a
 * rigid mesh with a position, an orientation quaternion and linear and
 * angular velocities; the states are the snapshot a step starts from).
 * pid: n caller ids (>= 0), mesh_id: their meshes, s: their states; all host
 * arrays, copied. Quaternions are normalised. The states are kept on the host
 * and, for ids below 2^24, in device memory for the device-side pair
 * preparation. A call waits for running queries that read the device copy.
 * Errors: MCD_E_INVALID (negative id, non-finite state, zero quaternion),
 * MCD_E_NOT_FOUND (unknown mesh). */
mcd_status mcd_particles_set(mcd_ctx* ctx, int32_t n, const int32_t* pid,
                             const int32_t* mesh_id, const mcd_state* s);

/* Submit a query over n particle pairs (pid_pairs: n*2 particle ids, host
 * array, copied). Static (o->dt == 0): per pair the minimum distance, its
 * closest points and the contact set {(i, j) : d_ij <= eps_a + eps_b}
 * (section 5, "Geometric model" and the contact-point definition). Time stamp
 * (o->dt > 0): per pair the first contact time in [0, dt], its status and the
 * contact set at that time (section 5, "Collision time detection", the case
 * distinctions and the widening remark: the time returned is the first one
 * known to be in contact). States and meshes are snapshot at submission
 * (lists of more than 4,096 pairs on up to 8 short-lived host threads).
 * Asynchronous; *ticket identifies the result. Errors: MCD_E_INVALID (bad
 * options, a pair repeating a particle), MCD_E_NOT_FOUND (unknown particle or
 * unloaded mesh), MCD_E_BUSY (the query exceeds the memory budget); the
 * error names the lowest bad pair. */
mcd_status mcd_query_pairs(mcd_ctx* ctx, int32_t n, const int32_t* pid_pairs,
                           const mcd_qopts* o, uint64_t* ticket);

/* Same query with the pair list in device memory (section 5, as
 * mcd_query_pairs): d_pairs holds n*2 int32 particle ids, caller-owned, and
 * must stay valid and unchanged until the ticket completes. `stream` (a
 * hipStream_t, or NULL for the context's stream) orders the read: the query
 * waits for the work queued on it before it reads the list; the call itself
 * does not block. The pairs are read and prepared on the device from the
 * device copies of the particle and mesh tables, so every particle id must
 * be below 2^24. Unknown ids, a pair repeating a particle or an unloaded mesh
 * make the ticket complete with MCD_E_NOT_FOUND / MCD_E_INVALID. Contact
 * records and pair results are as for mcd_query_pairs; mcd_fetch's pairs_out
 * returns the list as read. */
mcd_status mcd_query_pairs_dev(mcd_ctx* ctx, int32_t n, const int32_t* d_pairs,
                               const mcd_qopts* o, void* stream, uint64_t* ticket);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the static
 * MIXED contact query of mcd_query_pairs_dev, run synchronously on `stream`
 * (NULL: the context's stream), whose working memory is one fixed device
 * array of 143 MiB per GPU, held by the library until the process ends; the
 * call allocates nothing. d_pairs: n*2 int32 particle ids in device memory
 * (n <= 16384). d_results: n records in device memory, written as by
 * mcd_fetch. d_contacts: cap_contacts records in device memory, sorted by
 * (pair, tri_a, tri_b); *n_contacts (host, optional) receives the count, also
 * when cap_contacts is too small (MCD_E_INVALID). Queries beyond the array
 * (more than 2^24 tile pairs spanned, 2^20 kept by the cull, 2^22 near
 * triangle pairs, 2^19 FP64 candidates, or a pair with more than 4,096
 * contacts) fail with MCD_E_INVALID and the query must go through
 * mcd_query_pairs_dev. Calls in one process are serialised; calls that
 * overlapped on one GPU would race on the array. */
mcd_status mcd_query_pairs_noalloc(mcd_ctx* ctx, int32_t n, const int32_t* d_pairs, void* stream,
                                   mcd_pair_result* d_results, mcd_contact* d_contacts, int64_t cap_contacts,
                                   int64_t* n_contacts);

/* Cluster query (section 2, clustering: a cluster is a set of particles that
 * advance together): the library forms the candidate pairs inside the
 * cluster with the broad phase of mcd_broad_phase (checks 1 and 2 of section
 * 3; bounding spheres about the rotation centre, for dt > 0 swept along the
 * centre paths), on the device when every id is below 2^24, and runs the
 * pair query on them; pairs are ordered by the positions of both particles
 * in pid. Static cluster queries batch together. states: optional new states
 * for the n particles (all at the cluster's common time), or NULL. The
 * result adds the cluster's new time: the minimum toi over COLLIDES pairs,
 * else dt (mcd_cluster_time). Errors: MCD_E_INVALID (a particle listed
 * twice), MCD_E_NOT_FOUND (unknown particle), MCD_E_BUSY. */
mcd_status mcd_query_cluster(mcd_ctx* ctx, int32_t n, const int32_t* pid, const mcd_state* states,
                             const mcd_qopts* o, uint64_t* ticket);

/* Broad phase and clustering of a particle set (section 3: check 1, the
 * space-time bounding boxes of each particle's bounding sphere plus halo at
 * the start and the end of the step; check 2, the space-time tubes of those
 * spheres moving linearly over [0, dt], which must come within reach at a
 * common time; then the unconnected subgraphs of the resulting pair graph,
 * found by repeated min-labelling until nothing changes). pid: n particle ids
 * (host array, each once, ids below 2^24); dt >= 0 (0: static boxes and
 * spheres). Outputs, each optional (NULL to skip): cluster[i] the cluster of
 * pid[i], numbered 0.. in the order of each cluster's first member;
 * *n_clusters their count; pairs_out (2 * cap_pairs int32) the candidate
 * pairs as particle ids, ordered by the positions of both particles in pid;
 * *n_pairs their count (set even when cap_pairs is too small, which returns
 * MCD_E_INVALID). Runs on the device and returns when done; it waits for
 * running device-list queries first. Errors: MCD_E_INVALID, MCD_E_NOT_FOUND
 * (unknown id), MCD_E_HIP. */
mcd_status mcd_broad_phase(mcd_ctx* ctx, int32_t n, const int32_t* pid, double dt, int32_t* cluster,
                           int32_t* n_clusters, int32_t* pairs_out, int64_t cap_pairs, int64_t* n_pairs);

/* Options of the particle interaction solve (mcd_impulses). */
typedef struct {
    double restitution; /* e in [0, 1]: each contact's separation speed is driven to at least
                           max(0, -e u_n0), u_n0 its speed before the solve (0: the paper's
                           constraint that particles stop approaching) */
    double friction;    /* Coulomb coefficient mu >= 0 (0: frictionless) */
    double relax;       /* damping of the Picard updates, in (0, 1] (0 means 1) */
    double tol;         /* the iteration ends after a sweep whose largest change of a contact's
                           impulse is at most tol times the largest impulse (0 means 1e-4) */
    int32_t max_iter;   /* sweeps at most (0 means 100) */
    int32_t pad;
} mcd_impulse_opts;

/* Particle interaction (section 6, "Particle interaction": the impulses
 * exchanged at the contact points of a cluster so that particles in contact
 * stop approaching, by a Picard iteration that updates one contact point's
 * contribution at a time, with damped updates, Coulomb friction, and the
 * contact graph coloured so that contact points of one colour update in
 * parallel). Contact k joins particles pid_pairs[2k] (a) and pid_pairs[2k+1]
 * (b) at the point (pa + pb)/2 of contacts[k] (an mcd_contact record, e.g.
 * from a MCD_Q_FUSE query; only pa and pb are read), with normal pb - pa
 * (from a to b; when pa = pb, the line between the centres of mass). Masses
 * and inertia: each mesh as a closed solid of unit density (meshes that
 * enclose no volume are refused); velocities: the resident states
 * (mcd_particles_set), which the call does not change. The solve runs on the
 * device in one workgroup and returns when done.
 * Outputs: impulse (4n doubles: the normal impulse, then the tangential
 * impulse vector, world frame, per contact, acting on b; a takes the
 * opposite); pids_out (up to 2n ids: the particles in order of first
 * appearance) with *n_particles their count; vel_out (6 per particle: the new
 * v and w of its state); *sweeps the sweeps run. Any output may be NULL.
 * Errors: MCD_E_INVALID (n < 0, a null input, a pair repeating a particle,
 * options out of range, a mesh without volume), MCD_E_NOT_FOUND (unknown
 * particle id), MCD_E_HIP. */
mcd_status mcd_impulses(mcd_ctx* ctx, int32_t n, const int32_t* pid_pairs, const mcd_contact* contacts,
                        const mcd_impulse_opts* o, double* impulse, int32_t* n_particles, int32_t* pids_out,
                        double* vel_out, int32_t* sweeps);

/* Completion of an asynchronous query (the cluster tasks of section 2 finish
 * independently). mcd_poll sets *done to 1 when the ticket's results are
 * ready; MCD_E_NOT_FOUND for an unknown ticket. */
mcd_status mcd_poll(mcd_ctx* ctx, uint64_t ticket, int32_t* done);
/* Block until ready or timeout_ns (< 0: no limit). */
mcd_status mcd_wait(mcd_ctx* ctx, uint64_t ticket, int64_t timeout_ns);

/* Result sizes of a completed ticket. n_pairs: particle pairs (for cluster
 * queries, the candidate pairs the library formed). */
mcd_status mcd_result_sizes(mcd_ctx* ctx, uint64_t ticket, int32_t* n_pairs, int64_t* n_contacts);

/* Copy results into caller buffers: pr (cap_pairs entries) in query order,
 * contacts (cap_contacts) sorted by (pair, tri_a, tri_b). pairs_out (optional,
 * 2*cap_pairs int32) receives the particle ids of each pair. Any pointer may be
 * NULL to skip that part. Contact records beyond 4 MB are copied on up to 8
 * short-lived host threads. Fails with MCD_E_INVALID if a capacity is too
 * small. */
mcd_status mcd_fetch(mcd_ctx* ctx, uint64_t ticket, mcd_pair_result* pr, int32_t cap_pairs,
                     mcd_contact* contacts, int64_t cap_contacts, int32_t* pairs_out);

/* The results of a completed ticket without a copy (section 5, contact-point
 * definition, as mcd_fetch): pointers into the library's host memory (pinned
 * for the contact records of a single query), valid until mcd_release of the
 * ticket or mcd_destroy. Any output pointer may be NULL. *contacts is NULL for
 * a MCD_Q_DEVICE_OUT query and for a query without contact records. */
mcd_status mcd_result_view(mcd_ctx* ctx, uint64_t ticket, const mcd_pair_result** pr,
                           const mcd_contact** contacts, const int32_t** pairs);

/* Results of a completed MCD_Q_DEVICE_OUT query copied into caller device
 * memory (section 5, as mcd_fetch): d_pr (cap_pairs records) and d_contacts
 * (cap_contacts records, sorted by (pair, tri_a, tri_b)); either may be NULL.
 * The copies are queued on `stream` (a hipStream_t, NULL: the context's
 * stream) after the query's own work, and the call does not block; the caller
 * synchronises that stream before reading. mcd_release of the ticket waits for
 * the copies. MCD_E_INVALID if the query was not submitted with
 * MCD_Q_DEVICE_OUT or a capacity is too small. */
mcd_status mcd_fetch_dev(mcd_ctx* ctx, uint64_t ticket, mcd_pair_result* d_pr, int32_t cap_pairs,
                         mcd_contact* d_contacts, int64_t cap_contacts, void* stream);

/* New time of a completed cluster (or pair) query: minimum toi over pairs with
 * status COLLIDES, else dt (section 5, the update of t_new of a cluster; pairs
 * in contact at the start or moving apart do not constrain it). */
mcd_status mcd_cluster_time(mcd_ctx* ctx, uint64_t ticket, double* t_new);

/* Counters of a completed ticket (diagnostics; mcd_stats above). */
mcd_status mcd_query_stats(mcd_ctx* ctx, uint64_t ticket, mcd_stats* st);

/* Free a ticket's results; the ticket becomes unknown. */
mcd_status mcd_release(mcd_ctx* ctx, uint64_t ticket);

#ifdef __cplusplus
}
#endif

#endif /* MCD_H */
