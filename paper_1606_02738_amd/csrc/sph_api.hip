// C-ABI of libsph_hip: context lifetime, argument checks, stage ordering,
// statistics.
#include <math.h>
#include <string.h>

#include <new>

#include "sph_ctx.h"

thread_local Pool* g_pool = nullptr;

static const size_t POOL_ALIGN = 256;

void Pool::init(void* mem, size_t bytes)
{
    const uintptr_t a = ((uintptr_t)mem + POOL_ALIGN - 1) & ~(uintptr_t)(POOL_ALIGN - 1);
    base = (char*)a;
    size = bytes > (size_t)(a - (uintptr_t)mem) ? (bytes - (size_t)(a - (uintptr_t)mem)) & ~(POOL_ALIGN - 1) : 0;
    free_blocks.clear();
    if (size) free_blocks[0] = size;
    in_use = high = needed = 0;
}

void* Pool::take(size_t bytes)
{
    bytes = (bytes + POOL_ALIGN - 1) & ~(POOL_ALIGN - 1);
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, len = it->second;
        free_blocks.erase(it);
        if (len > bytes) free_blocks[off + bytes] = len - bytes;
        in_use += bytes;
        high = std::max(high, in_use);
        return base + off;
    }
    needed = std::max(needed, in_use + bytes);
    return nullptr;
}

void Pool::give(void* p, size_t bytes)
{
    bytes = (bytes + POOL_ALIGN - 1) & ~(POOL_ALIGN - 1);
    size_t off = (size_t)((char*)p - base), len = bytes;
    in_use -= bytes;
    auto nx = free_blocks.lower_bound(off);
    if (nx != free_blocks.end() && off + len == nx->first) {
        len += nx->second;
        nx = free_blocks.erase(nx);
    }
    if (nx != free_blocks.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            off = pv->first;
            len += pv->second;
            free_blocks.erase(pv);
        }
    }
    free_blocks[off] = len;
}

sph_status buf_ensure(DevBuf& b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return SPH_OK;
    Pool* pool = b.pool ? b.pool : g_pool;
    if (!pool) return SPH_ERR_STATE;  // no workspace in scope
    buf_free(b);
    const size_t want = (bytes + bytes / 8 + 256 + POOL_ALIGN - 1) & ~(POOL_ALIGN - 1);
    void* p = pool->take(want);
    if (!p) {
        p = pool->take(bytes);  // without the growth slack
        if (!p) return SPH_ERR_WORKSPACE;
        b.cap = (bytes + POOL_ALIGN - 1) & ~(POOL_ALIGN - 1);
    } else {
        b.cap = want;
    }
    b.p = p;
    b.pool = pool;
    return SPH_OK;
}

void buf_free(DevBuf& b)
{
    if (b.p && b.pool) b.pool->give(b.p, b.cap);
    b.p = nullptr;
    b.cap = 0;
    b.pool = nullptr;
}

extern "C" {

const char* sph_status_str(sph_status s)
{
    switch (s) {
    case SPH_OK: return "ok";
    case SPH_ERR_INVALID: return "invalid argument or input";
    case SPH_ERR_HIP: return "HIP runtime error";
    case SPH_ERR_NOT_CONVERGED: return "smoothing lengths not converged";
    case SPH_ERR_H_EXCEEDS_CELL: return "smoothing length exceeds the cell grid";
    case SPH_ERR_BOX_TOO_SMALL: return "smoothing length exceeds a third of the box";
    case SPH_ERR_WORKSPACE: return "workspace too small";
    case SPH_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

const char* sph_version(void) { return "libsph_hip 0.1 gfx950 wave64"; }

// Workspace estimate: fixed part plus bytes per particle of every buffer the
// stages keep (keys and permutation, kernel-side particle data, iteration
// brackets, octree and leaf arrays, cell lists, the sort stage's orders, the
// predictor's features and samples of up to n / 8 particles, interpolation
// at up to n points; particle lists when selected).
static size_t workspace_estimate(const sph_params& p, int64_t n)
{
    const bool f64 = p.precision == SPH_FP64;
    size_t per = f64 ? 768 : 640;
    if (p.lists == SPH_LISTS_PARTICLE) per += f64 ? 2048 : 1536;
    return ((size_t)64 << 20) + (size_t)n * per + (size_t)p.n_domains * 4096;
}

sph_status sph_workspace_size(const sph_params* params, int64_t n, size_t* bytes)
{
    if (!params || !bytes || n < 1 || n >= ((int64_t)1 << 31)) return SPH_ERR_INVALID;
    if (params->n_domains < 1) return SPH_ERR_INVALID;
    *bytes = workspace_estimate(*params, n);
    return SPH_OK;
}

sph_status sph_create(const sph_params* params, void* workspace, size_t bytes, void* hip_stream, sph_ctx** out)
{
    if (!params || !out) return SPH_ERR_INVALID;
    *out = nullptr;
    if (!workspace || bytes < SPH_WORKSPACE_MIN) return SPH_ERR_INVALID;
    const sph_params& p = *params;
    if (p.n_domains < 1 || !p.boxes) return SPH_ERR_INVALID;
    if (!(p.gamma > 1.0) || !(p.eta > 0.0) || !(p.kernel_gamma > 0.0) || !(p.h_tol > 0.0)) return SPH_ERR_INVALID;
    if (p.max_h_iter < 1 || p.n_split < 1 || p.n_split > SPH_MAX_LEAF) return SPH_ERR_INVALID;
    if (p.precision < SPH_FP64 || p.precision > SPH_FP32) return SPH_ERR_INVALID;
    if (p.exec_mode < SPH_EXEC_GRID || p.exec_mode > SPH_EXEC_PERSISTENT) return SPH_ERR_INVALID;
    if (p.prune < SPH_PRUNE_BOX || p.prune > SPH_PRUNE_SORTED) return SPH_ERR_INVALID;
    if (p.use_graph < 0 || p.use_graph > 1) return SPH_ERR_INVALID;
    if (p.rebuild_steps < 0 || p.rebuild_steps > 1000) return SPH_ERR_INVALID;
    if (p.h_drift != 0 && p.h_drift != 1) return SPH_ERR_INVALID;
    if (p.force_mode != SPH_FORCE_PAIRS && p.force_mode != SPH_FORCE_GATHER) return SPH_ERR_INVALID;
    if (p.force_mode == SPH_FORCE_GATHER && p.prune != SPH_PRUNE_BOX) return SPH_ERR_INVALID;
    if (p.lists != SPH_LISTS_CELL && p.lists != SPH_LISTS_PARTICLE) return SPH_ERR_INVALID;
    if (p.lists == SPH_LISTS_PARTICLE && p.force_mode != SPH_FORCE_GATHER) return SPH_ERR_INVALID;
    if (p.tile != 0 && p.tile != 256 && p.tile != 512 && p.tile != 1024) return SPH_ERR_INVALID;
    for (int wv : {p.waves_density, p.waves_force})
        if (wv != 0 && wv != 4 && wv != 5 && wv != 6 && wv != 8) return SPH_ERR_INVALID;
    if (p.batch != 0 && p.batch != 16 && p.batch != 32) return SPH_ERR_INVALID;
    for (int k = 0; k < 3 * p.n_domains; k++)
        if (!(p.boxes[k] > 0.0) || !isfinite(p.boxes[k])) return SPH_ERR_INVALID;
    sph_ctx* c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_ERR_INVALID;
    c->pool.init(workspace, bytes);
    PoolScope ps(&c->pool);
    c->prm = p;
    c->boxes.assign(p.boxes, p.boxes + 3 * p.n_domains);
    c->prm.boxes = nullptr;
    c->stream = (hipStream_t)hip_stream;
    sph_status s = SPH_OK;
    if (s == SPH_OK) s = buf_ensure(c->flags, FI_NFLAGS * sizeof(int));
    if (s == SPH_OK) s = buf_ensure(c->counters, CNT_ALLOC * 8);
    if (s == SPH_OK) s = buf_ensure(c->dparam, 8 * sizeof(double));
    if (s == SPH_OK && hipMemsetAsync(c->dparam.p, 0, 8 * sizeof(double), c->stream) != hipSuccess) s = SPH_ERR_HIP;
    if (s == SPH_OK) s = buf_ensure(c->dom_d, (size_t)p.n_domains * sizeof(DomainInfo));
    if (s == SPH_OK) s = buf_ensure(c->dstat, (size_t)p.n_domains * 24);
    for (int k = 0; k < 8 && s == SPH_OK; k++)
        if (hipEventCreate(&c->ev[k]) != hipSuccess) s = SPH_ERR_HIP;
    for (int k = 0; k < 4 && s == SPH_OK; k++)
        if (hipEventCreate(&c->kev[k]) != hipSuccess) s = SPH_ERR_HIP;
    // a second stream for the build's permutation (optional: without it the
    // permutation stays on the caller's stream)
    if (s == SPH_OK) {
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->side_ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->side_ev[1], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (c->side) (void)hipStreamDestroy(c->side);
            for (hipEvent_t& e : c->side_ev)
                if (e) (void)hipEventDestroy(e), e = nullptr;
            c->side = nullptr;
        }
    }
    if (s == SPH_OK && hipMemsetAsync(c->flags.p, 0, FI_NFLAGS * sizeof(int), c->stream) != hipSuccess) s = SPH_ERR_HIP;
    if (s == SPH_OK && hipMemsetAsync(c->counters.p, 0, CNT_ALLOC * 8, c->stream) != hipSuccess) s = SPH_ERR_HIP;
    if (s != SPH_OK) {
        sph_destroy(c);
        return s;
    }
    *out = c;
    return SPH_OK;
}

sph_status sph_destroy(sph_ctx* c)
{
    if (!c) return SPH_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    for (hipEvent_t e : c->side_ev)
        if (e) (void)hipEventDestroy(e);
    DevBuf* all[] = {&c->dom_d, &c->dstat, &c->keys[0], &c->keys[1], &c->vals[0], &c->vals[1], &c->ikeys[0], &c->ikeys[1], &c->ivals[0], &c->ivals[1], &c->dranges, &c->tmp, &c->nodes, &c->wnodes,
                     &c->nchild, &c->coff, &c->lvl_cmap, &c->lvl_bnd, &c->leafmark, &c->leafscan, &c->leaf_node, &c->l_begin, &c->l_count,
                     &c->l_origin, &c->l_lo, &c->l_hi, &c->l_hlist, &c->l_dom, &c->l_off, &c->l_active, &c->l_sorted,
                     &c->l_cnt, &c->list, &c->pos4, &c->fv4, &c->hf, &c->skey, &c->sidx,
                     &c->hlo, &c->hhi, &c->conv, &c->flags, &c->counters,
                     &c->scan_tmp, &c->rs_hist, &c->sums, &c->dsum_part, &c->fgrid, &c->fcount, &c->mlp_X, &c->mlp_hprev, &c->mlp_params, &c->mlp_packed, &c->mlp_m, &c->mlp_v, &c->ds_count, &c->dparam, &c->walk_scratch, &c->walk_ovf, &c->walk_link,
                     &c->pq, &c->pR, &c->plist, &c->prem, &c->plen, &c->pskin, &c->pq0, &c->pext, &c->pbox,
                     &c->ch_base, &c->ch_p0, &c->ch_n, &c->ch_uo, &c->ch_ro, &c->ch_U};
    for (DevBuf* b : all) buf_free(*b);
    for (int k = 0; k < 8; k++)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    for (int k = 0; k < 4; k++)
        if (c->kev[k]) (void)hipEventDestroy(c->kev[k]);
    for (int k = 0; k < 2; k++)
        if (c->pev[k]) (void)hipEventDestroy(c->pev[k]);
    if (c->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)c->graph_exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return SPH_OK;
}

sph_status sph_build_cells(sph_ctx* c, const sph_particles* p)
{
    if (!c || !p) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (p->n <= 0 || p->n >= (int64_t)1 << 31) return SPH_ERR_INVALID;
    const double* req[] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->u, p->m, p->H,
                           p->rho, p->drho_dH, p->ax, p->ay, p->az, p->dudt};
    for (const double* a : req)
        if (!a) return SPH_ERR_INVALID;
    if (c->prm.n_domains > 1 && !p->domain) return SPH_ERR_INVALID;
    c->P = *p;
    c->n = p->n;
    c->bound = true;
    c->built = c->sorted = c->dens_done = c->ghost_done = c->force_done = false;
    c->mlp_pending = false;
    SPH_CHECK_HIP(hipEventRecord(c->ev[6], c->stream));
    sph_status s = build_all(c);
    if (s == SPH_OK) c->st.rebuilds++;
    return s;
}

sph_status sph_sort_cells(sph_ctx* c)
{
    if (!c) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->built) return SPH_ERR_STATE;
    SPH_TRY(sort_all(c));
    SPH_CHECK_HIP(hipEventRecord(c->ev[7], c->stream));
    return SPH_OK;
}

sph_status sph_density(sph_ctx* c)
{
    if (!c) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->sorted) return SPH_ERR_STATE;
    return density_all(c);
}

sph_status sph_ghost(sph_ctx* c)
{
    if (!c) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    return ghost_all(c);
}

sph_status sph_force(sph_ctx* c)
{
    if (!c) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    return force_all(c);
}

sph_status sph_density_ghost_force(sph_ctx* c)
{
    if (!c) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->sorted) return SPH_ERR_STATE;
    c->predicted = false;
    if (c->prm.use_graph) return dgf_graph(c);
    SPH_TRY(density_all(c));
    SPH_TRY(ghost_all(c));
    return force_all(c);
}

sph_status sph_step(sph_ctx* c, double dt)
{
    if (!c) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!(dt > 0.0) || !isfinite(dt)) return SPH_ERR_INVALID;
    if (!c->force_done) return SPH_ERR_STATE;
    return step_all(c, dt);
}

static double elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0;
    }
    return ms;
}

sph_status sph_get_stats(sph_ctx* c, sph_stats* out)
{
    if (!c || !out) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    unsigned long long hc[CNT_ALLOC];
    SPH_CHECK_HIP(hipMemcpyAsync(hc, c->counters.p, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
    std::vector<double> sums;
    if (c->sums_pending && c->sums_dev) {
        sums.resize((size_t)c->prm.n_domains * 5);
        SPH_CHECK_HIP(hipMemcpyAsync(sums.data(), c->sums_dev, sums.size() * 8, hipMemcpyDeviceToHost, c->stream));
    }
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    if (c->force_pending) {
        // the gather forms count every pair from both sides
        c->st.n_force = (int64_t)(c->prm.force_mode == SPH_FORCE_GATHER ? hc[CNT_NFORCE] / 2 : hc[CNT_NFORCE]);
        c->st.n_dens = (int64_t)hc[CNT_NDENS_F];  // exact at the final H
        c->st.t_force_kernel_ms = elapsed(c->kev[2], c->kev[3]);
        c->force_pending = false;
    }
    if (!sums.empty()) {
        for (int k = 0; k < 5; k++) {
            double t = 0.0;
            for (int d = 0; d < c->prm.n_domains; d++) t += sums[5 * d + k];
            c->st.conserved[k] = t;
        }
        c->sums_pending = false;
    }
    const unsigned long long nf = hc[CNT_NFORCE_SUM];
    c->st.n_force_total = (int64_t)(c->prm.force_mode == SPH_FORCE_GATHER ? nf / 2 : nf);
    c->st.n_dens_total = (int64_t)hc[CNT_NDENS_SUM];
    c->st.force_calls = (int64_t)hc[CNT_FORCE_CALLS];
    c->st.n = c->n;
    c->st.n_leaves = c->n_leaves;
    c->st.n_nodes = c->n_nodes;
    c->st.n_list = c->n_list;
    if (c->built && !c->pair_tasks_valid) {
        SPH_TRY(count_pair_tasks(c));
        unsigned long long np = 0;
        SPH_CHECK_HIP(hipMemcpyAsync(&np, (unsigned long long*)c->counters.p + CNT_NPAIR, 8, hipMemcpyDeviceToHost,
                                     c->stream));
        SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
        c->st.n_pair_tasks = (int64_t)np;
        c->pair_tasks_valid = true;
    } else if (!c->built) {
        c->st.n_pair_tasks = 0;
    }
    c->st.depth = c->depth;
    c->st.key_bits = c->key_bits;
    c->st.t_density_ms = c->dens_done ? elapsed(c->ev[0], c->ev[1]) : -1.0;
    c->st.t_ghost_ms = c->ghost_done ? elapsed(c->ev[2], c->ev[3]) : -1.0;
    c->st.t_force_ms = c->force_done ? elapsed(c->ev[4], c->ev[5]) : -1.0;
    c->st.t_build_ms = c->sorted ? elapsed(c->ev[6], c->ev[7]) : -1.0;
    c->st.t_predict_ms = c->pev_done ? elapsed(c->pev[0], c->pev[1]) : -1.0;
    c->st.steps_since_build = c->steps_since_build;
    c->st.n_builds = c->n_builds;
    c->st.list_margin = c->margin_h;
    c->st.n_chunks = c->n_chunks;
    c->st.n_plist = c->n_plist;
    c->st.n_union = c->n_union;
    c->st.workspace_bytes = (int64_t)c->pool.size;
    c->st.workspace_in_use = (int64_t)c->pool.in_use;
    c->st.workspace_high = (int64_t)c->pool.high;
    c->st.workspace_needed = (int64_t)c->pool.needed;
    *out = c->st;
    return SPH_OK;
}

sph_status sph_domain_sums(sph_ctx* c, double* out)
{
    if (!c || !out) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->built) return SPH_ERR_STATE;
    return domain_sums(c, out);
}

}  // extern "C"
