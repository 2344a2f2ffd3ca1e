// Host-side context of libsph_hip and the launch wrappers shared by the
// translation units.  Not part of the C-ABI.
#pragma once

#include <map>
#include <vector>

#include "sph_internal.h"

// Device memory of the library: blocks carved from a caller-owned workspace
// (first fit over a free list, neighbours merged on release).  The library
// itself never allocates device memory.
struct Pool {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes
    size_t in_use = 0, high = 0;
    size_t needed = 0;  // in-use bytes plus the request that did not fit (0: none failed)
    void init(void* mem, size_t bytes);
    void* take(size_t bytes);
    void give(void* p, size_t bytes);
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Pool* pool = nullptr;
};

// The pool the calls on this host thread carve from: set by every C-ABI entry
// point for its duration (the context's pool, or one over the workspace a
// context-free call is given).
extern thread_local Pool* g_pool;
struct PoolScope {
    Pool* prev;
    explicit PoolScope(Pool* p) : prev(g_pool) { g_pool = p; }
    ~PoolScope() { g_pool = prev; }
};

struct sph_ctx {
    sph_params prm;
    Pool pool;                   // over the caller's workspace
    std::vector<double> boxes;   // n_domains x 3
    hipStream_t stream = nullptr;

    // bound particles
    sph_particles P{};
    bool bound = false;
    int64_t n = 0;

    // domains and key layout
    std::vector<DomainInfo> dom_h;
    int n_top_total = 0;
    int D = 0;                   // octree levels encoded in the key
    int key_bits = 0;
    double min_s0 = 0;           // smallest top-cell edge over all boxes

    // octree / leaves / lists
    int n_nodes = 0, n_leaves = 0, depth = 0;
    int max_leaf = 0;            // particles in the fullest leaf
    int64_t n_list = 0;
    bool pair_tasks_valid = false;  // the device count of pair tasks belongs to the current lists
    std::vector<int> level_off;  // node index of the first node of each level

    // stage state
    bool built = false, sorted = false, dens_done = false, ghost_done = false, force_done = false;
    bool in_step = false;  // inside sph_step (the refresh of the next step checks the FP32 extent rule)
    bool predicted = false;      // ghost/force use the predicted v, u of a step
    double hdt_h = 0.0;          // half the step in progress (the prediction's interval)
    double hdt_up = 0.0;         // source of the upload of the prediction's half step

    // counters of the last calls
    sph_stats st{};
    bool force_pending = false;   // the last force call's counts are still on the device
    bool sums_pending = false;    // the last step's FP64 totals are still on the device
    const double* sums_dev = nullptr;
    unsigned long long stale_h[2] = {0, 0};

    // device buffers
    DevBuf dom_d, dstat;          // DomainInfo[], per-domain (hmax, hmin) as u64 bits and particle count
    DevBuf keys[2], vals[2];      // radix sort ping-pong
    DevBuf ikeys[2], ivals[2];    // interpolation point-order sort ping-pong
    DevBuf dranges;               // per-box particle ranges [n_domains + 1]
    const void* keys_sorted = nullptr;  // sorted Morton keys of the last build
    DevBuf tmp;                   // permutation scratch (8 B per particle)
    DevBuf nodes, nchild, coff;   // octree; per level: children, chunk offsets
    DevBuf lvl_cmap, lvl_bnd;     // per level: chunk -> cell, octant bounds (9 per cell)
    DevBuf wnodes;                // compact cells for the list walk
    DevBuf leafmark, leafscan;    // per particle
    DevBuf leaf_node;             // leaf -> node
    DevBuf l_begin, l_count, l_origin, l_lo, l_hi, l_hlist, l_dom, l_off, l_active, l_sorted, l_cnt;
    DevBuf list;
    DevBuf walk_scratch;          // per-leaf slots of the one-pass list walk
    DevBuf walk_ovf, walk_link;   // its overflow chunks; chunk links (head, incomplete, next)
    int walk_cap = 128;           // entries per slot (grows after an overflow)
    bool dens_outputs_dead = false;  // the build need not permute rho, drho_dH, omega, P
    bool radii_fresh = false;        // list radii and walk bounds are those of the current H
    hipStream_t side = nullptr;      // second stream of the build (permutation), default priority
    hipEvent_t side_ev[2] = {};      // sort done (context stream), permutation done (second stream)
    bool side_pending = false;       // the context stream has not yet waited for side_ev[1]
    DevBuf pos4, fv4, hf;         // kernel-side particle data (T = float or double)
    // per-particle lists (lists = SPH_LISTS_PARTICLE)
    DevBuf pq, pR, plen, plist;   // fixed-point positions + mass, list radii, list lengths, entries
    DevBuf prem;                  // FP32 modes: remainders of the fixed-point coordinates
    DevBuf pskin, pq0, pext, pbox;  // skins, fixed-point positions at the build, extents R + s,
                                    // per-box largest R and s
    double list_dt = 0.0;         // step length of the build's step (0: a build outside a step)
    double skin_max = 0.0;        // largest skin of the last build
    DevBuf ch_base, ch_p0, ch_n;  // chunks: first chunk of each leaf; first particle, count
    DevBuf ch_uo, ch_ro, ch_U;    // union offsets, row offsets, union members
    int n_chunks = 0;
    int plist_rows = 0;           // rows of the current particle lists
    int64_t n_union = 0;          // union members over all chunks
    bool plist_valid = false;
    int64_t n_plist = 0;          // entries of the current particle lists
    DevBuf skey, sidx;            // per-direction sorted projections
    DevBuf hlo, hhi, conv;        // Newton brackets and converged flags
    DevBuf flags, counters;       // device flags (int[64], see FI_*) and counters (int64)
    DevBuf scan_tmp;              // scan block sums
    DevBuf rs_hist;               // radix-sort digit histograms
    DevBuf sums;                  // per-domain FP64 conservation partials
    DevBuf dsum_part;

    hipEvent_t ev[8] = {};
    void* graph_exec = nullptr;        // hipGraphExec_t of the density-ghost-force graph
    std::vector<uint8_t> graph_key;    // launch arguments it was captured with
    hipStream_t cap_stream = nullptr;  // private stream used only for capture
    hipEvent_t kev[4] = {};     // per-launch kernel timing

    // lazy rebuild: displacement since the build and the list skin
    DevBuf dparam;                      // double[8]: [0] list margin (2 x displacement), [1] max speed (bits),
                                        // [2] half step of the ghost's prediction (0: none)
    double delta = 0.0;                 // largest displacement bound since the build
    double skin_abs = 0.0;              // absolute list skin of the last build
    double margin_h = 0.0;              // host copy of dparam[0] (source of its uploads)
    int64_t steps_since_build = 0, n_builds = 0;

    // learned H predictor
    std::vector<FeatGrid> fgrid_h;
    int64_t fgrid_n = -1, fgrid_cells = 0;
    DevBuf fgrid, fcount;               // FeatGrid[], per-cell counts
    DevBuf mlp_X, mlp_hprev;            // features and previous H of the current step (particle order)
    DevBuf mlp_params, mlp_packed, mlp_m, mlp_v;
    float* ds_X = nullptr;              // recorded samples (the caller's buffers)
    float* ds_y = nullptr;
    DevBuf ds_count;
    bool rec_on = false, h_pred = false, mlp_ready = false, mlp_have = false, mlp_pending = false;
    int64_t rec_cap = 0;
    double rec_rate = 0.0;
    uint64_t rec_seed = 0;
    int adam_t = 0;
    int64_t step_count = 0;
    hipEvent_t pev[2] = {};             // timing of the predictor stage of the last step
    bool pev_done = false;

    int elem_size() const { return prm.precision == SPH_FP64 ? 8 : 4; }
};

// buffer management (sph_api.hip)
sph_status buf_ensure(DevBuf& b, size_t bytes);
void buf_free(DevBuf& b);

#define SPH_CHECK_HIP(expr)                                  \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return SPH_ERR_HIP;            \
    } while (0)
#define SPH_CHECK_LAUNCH() SPH_CHECK_HIP(hipGetLastError())
#define SPH_TRY(expr)                                        \
    do {                                                     \
        sph_status _s = (expr);                              \
        if (_s != SPH_OK) return _s;                         \
    } while (0)

// primitives (sph_prims.hip)
// Exclusive scan of n int32 values (in may equal out); *d_total (device) = sum.
sph_status scan_exclusive(sph_ctx* c, const int* in, int* out, int n, int* d_total);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits between
// the ping-pong buffers kb[0..1] / vb[0..1] (input in [0]); the sorted data
// ends in kb[res]/vb[res], res returned through *res_idx.
sph_status radix_sort(sph_ctx* c, int n, int bits, DevBuf* kb, DevBuf* vb, int* res_idx);

// build stages (sph_build.hip)
sph_status build_all(sph_ctx* c);
sph_status sort_all(sph_ctx* c);
sph_status relist(sph_ctx* c);
sph_status count_pair_tasks(sph_ctx* c);
sph_status node_hmax_all(sph_ctx* c, bool set_hlist);
sph_status refresh_leaves(sph_ctx* c, bool* fresh);
sph_status domain_ranges(sph_ctx* c);

// per-particle lists (sph_plist.hip)
struct DensArgs;
sph_status plist_build(sph_ctx* c);
sph_status plist_ext(sph_ctx* c, bool final, double* boxmax_host);
sph_status plist_refresh(sph_ctx* c, bool* fresh);
sph_status launch_density_plist(sph_ctx* c, const DensArgs& d);
sph_status launch_force_plist(sph_ctx* c, const int* gate);

// interaction stages (sph_interact.hip)
sph_status density_all(sph_ctx* c);
sph_status ghost_all(sph_ctx* c);
sph_status force_all(sph_ctx* c);
sph_status step_all(sph_ctx* c, double dt);
sph_status dgf_graph(sph_ctx* c);

// learned H predictor (sph_mlp.hip)
sph_status mlp_features(sph_ctx* c, double dt, float* X, double* hprev);
sph_status mlp_pre_build(sph_ctx* c, double dt);
sph_status mlp_post_step(sph_ctx* c);
sph_status domain_sums(sph_ctx* c, double* host_out);
