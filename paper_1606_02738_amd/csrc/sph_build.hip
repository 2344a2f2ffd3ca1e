// Cell construction and sort stage (Sec. 3.1 of the paper): top-level grid
// of cells of edge >= the largest smoothing length, Morton keys, radix sort,
// recursive octree split of cells holding more than n_split particles,
// leaf cells, neighbour-cell lists between leaves within range, and the
// per-direction sorted projections used to prune pair candidates.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sph_ctx.h"

// ---------------------------------------------------------------------------
// Validation: finite inputs, positive m and H, positions inside [0,L) of the
// particle's box; per-box largest and smallest H.
// ---------------------------------------------------------------------------
__device__ inline void flush_hrange(unsigned long long* dstat, int d, double hmx, double hmn, unsigned long long cnt)
{
    atomicMax(&dstat[3 * d], (unsigned long long)__double_as_longlong(hmx));
    atomicMin(&dstat[3 * d + 1], (unsigned long long)__double_as_longlong(hmn));
    atomicAdd(&dstat[3 * d + 2], cnt);
}

// Each workgroup takes one contiguous range of particles (coalesced within
// it); each thread keeps the H range of its current box and flushes it when
// the box changes, which happens only where a range crosses from one box
// to the next when the particles are grouped by box (the generators' order
// and the Morton order after a build); at the end a wave whose lanes share
// one box reduces across lanes first (one atomic pair per wave).  (A
// grid-stride loop would change box at almost every step for many boxes
// and serialise on the per-box atomics.)
__global__ __launch_bounds__(256) void k_validate(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                                  const double* __restrict__ z, const double* __restrict__ H,
                                                  const double* __restrict__ m, const int32_t* __restrict__ dom,
                                                  int ndom, const DomainInfo* __restrict__ di,
                                                  unsigned long long* dstat, int* flags)
{
    int dcur = -1;
    double hmx = 0.0, hmn = INFINITY;
    unsigned long long cnt = 0;
    bool bad = false;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(n, b0 + per);
    // four particles per thread and round, their loads issued together
    constexpr int U = 4;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += U * blockDim.x) {
        double px[U], py[U], pz[U], h[U], mm[U];
        int d[U];
        for (int u = 0; u < U; u++) {
            const int64_t j = min(i + (int64_t)u * blockDim.x, b1 - 1);
            d[u] = dom ? dom[j] : 0;
            px[u] = x[j];
            py[u] = y[j];
            pz[u] = z[j];
            h[u] = H[j];
            mm[u] = m[j];
        }
        for (int u = 0; u < U; u++) {
            if (i + (int64_t)u * blockDim.x >= b1) break;
            if (d[u] < 0 || d[u] >= ndom) {
                bad = true;
                continue;
            }
            const double* L = di[d[u]].L;
            const bool good = isfinite(px[u]) && isfinite(py[u]) && isfinite(pz[u]) && px[u] >= 0.0 && px[u] < L[0] &&
                              py[u] >= 0.0 && py[u] < L[1] && pz[u] >= 0.0 && pz[u] < L[2] && isfinite(h[u]) &&
                              h[u] > 0.0 && isfinite(mm[u]) && mm[u] > 0.0;
            if (!good) {
                bad = true;
                continue;
            }
            if (d[u] != dcur) {
                if (dcur >= 0) flush_hrange(dstat, dcur, hmx, hmn, cnt);
                dcur = d[u];
                hmx = 0.0;
                hmn = INFINITY;
                cnt = 0;
            }
            hmx = fmax(hmx, h[u]);
            hmn = fmin(hmn, h[u]);
            cnt++;
        }
    }
    if (bad) atomicOr(flags, FLAG_INVALID);
    // all lanes of a wave on one box: reduce across the wave, and across the
    // workgroup when its four waves share that box (one atomic triple per
    // workgroup: all of them meet on the same address when there is one box)
    __shared__ int wd[4];
    __shared__ double wmx[4], wmn[4];
    __shared__ unsigned long long wcnt[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int d0 = __shfl(dcur, 0);
    const bool uni = __ballot(dcur != d0) == 0ull;
    if (uni && d0 >= 0) {
        for (int off = 32; off > 0; off >>= 1) {
            hmx = fmax(hmx, __shfl_xor(hmx, off));
            hmn = fmin(hmn, __shfl_xor(hmn, off));
            cnt += __shfl_xor(cnt, off);
        }
    }
    if (lane == 0) {
        wd[w] = uni ? d0 : -2;  // -2: the wave flushes lane by lane
        wmx[w] = hmx;
        wmn[w] = hmn;
        wcnt[w] = cnt;
    }
    __syncthreads();
    const int db = wd[0];
    const bool block_uni = db >= 0 && wd[1] == db && wd[2] == db && wd[3] == db && blockDim.x == 256;
    if (block_uni) {
        if (threadIdx.x == 0)
            flush_hrange(dstat, db, fmax(fmax(wmx[0], wmx[1]), fmax(wmx[2], wmx[3])),
                         fmin(fmin(wmn[0], wmn[1]), fmin(wmn[2], wmn[3])), wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3]);
    } else if (uni && d0 >= 0) {
        if (lane == 0) flush_hrange(dstat, d0, hmx, hmn, cnt);
    } else if (dcur >= 0) {
        flush_hrange(dstat, dcur, hmx, hmn, cnt);
    }
}

__device__ inline uint64_t spread3(uint32_t v, int bits)
{
    uint64_t r = 0;
    for (int b = 0; b < bits; b++) r |= (uint64_t)((v >> b) & 1u) << (3 * b);
    return r;
}

__device__ inline int top_coord(double x, double s0, int nt)
{
    int ix = (int)floor(x / s0);
    return ix < 0 ? 0 : (ix >= nt ? nt - 1 : ix);
}

// Morton key: global top-cell index in the high bits, D interleaved bits per
// dimension of the position inside the top cell below.
__global__ __launch_bounds__(256) void k_keys(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, const int32_t* __restrict__ dom,
                                              const DomainInfo* __restrict__ di, int D, uint64_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DomainInfo& I = di[dom ? dom[i] : 0];
    const double p[3] = {x[i], y[i], z[i]};
    int t[3];
    uint32_t q[3];
    const double scale = (double)(1u << D);
    for (int a = 0; a < 3; a++) {
        t[a] = top_coord(p[a], I.s0[a], I.n_top[a]);
        double f = (p[a] - t[a] * I.s0[a]) / I.s0[a] * scale;
        long qi = (long)floor(f);
        if (qi < 0) qi = 0;
        if (qi > (1l << D) - 1) qi = (1l << D) - 1;
        q[a] = (uint32_t)qi;
    }
    const uint64_t top = (uint64_t)I.top_offset + ((uint64_t)t[0] * I.n_top[1] + t[1]) * I.n_top[2] + t[2];
    keys[i] = (top << (3 * D)) | (spread3(q[0], D) << 2) | (spread3(q[1], D) << 1) | spread3(q[2], D);
    vals[i] = (uint32_t)i;
}

struct FeatRow {
    float4 a, b;  // one row of predictor features (SPH_MLP_XSTRIDE floats)
};
static_assert(sizeof(FeatRow) == SPH_MLP_XSTRIDE * sizeof(float), "feature row");

// dst[i] = src[perm[i]]: four consecutive i per thread, so that four
// independent loads are in flight (perm is 16-byte aligned).
template <typename V>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const uint32_t* __restrict__ perm, const V* __restrict__ src,
                                                V* __restrict__ dst)
{
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 + 4 <= n) {
        const uint4 p = *(const uint4*)(perm + i0);
        const V a = src[p.x], b = src[p.y], c = src[p.z], d = src[p.w];
        dst[i0] = a;
        dst[i0 + 1] = b;
        dst[i0 + 2] = c;
        dst[i0 + 3] = d;
    } else {
        for (int64_t i = i0; i < n; i++) dst[i] = src[perm[i]];
    }
}

// dst[i] = src[i] for n 8-byte elements, 32 bytes per thread (both buffers
// 16-byte aligned).
__global__ __launch_bounds__(256) void k_copy8(int64_t n, const uint64_t* __restrict__ src, uint64_t* __restrict__ dst)
{
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 + 4 <= n) {
        const uint4 a = *(const uint4*)(src + i0), b = *(const uint4*)(src + i0 + 2);
        *(uint4*)(dst + i0) = a;
        *(uint4*)(dst + i0 + 2) = b;
    } else {
        for (int64_t i = i0; i < n; i++) dst[i] = src[i];
    }
}

__device__ inline int lower_bound_u64(const uint64_t* a, int lo, int hi, uint64_t v)
{
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Level-0 cells: the top grid of every box.
__global__ __launch_bounds__(256) void k_top_nodes(int n_top_total, int ndom, const DomainInfo* __restrict__ di,
                                                   const uint64_t* __restrict__ keys, int n, int D, Node* nodes)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_top_total) return;
    int d = 0;
    while (d + 1 < ndom && di[d + 1].top_offset <= t) d++;
    const DomainInfo& I = di[d];
    const int loc = t - I.top_offset;
    const int tz = loc % I.n_top[2], ty = (loc / I.n_top[2]) % I.n_top[1], tx = loc / (I.n_top[2] * I.n_top[1]);
    Node nd;
    nd.key_lo = (uint64_t)t << (3 * D);
    nd.begin = lower_bound_u64(keys, 0, n, nd.key_lo);
    nd.count = lower_bound_u64(keys, nd.begin, n, (uint64_t)(t + 1) << (3 * D)) - nd.begin;
    nd.first_child = -1;
    nd.n_child = 0;
    nd.level = 0;
    nd.domain = d;
    nd.leaf = -1;
    nd.top = t;
    nd.c_lo[0] = tx * I.s0[0]; nd.c_lo[1] = ty * I.s0[1]; nd.c_lo[2] = tz * I.s0[2];
    for (int a = 0; a < 3; a++) {
        nd.c_sz[a] = I.s0[a];
        nd.lo[a] = INFINITY;
        nd.hi[a] = -INFINITY;
    }
    nd.hmax = 0.0;
    nd.hmin = INFINITY;
    nd.merged = 0;
    nd.pad = 0;
    nodes[t] = nd;
}

// Children of a split cell: octants holding more than n_split particles
// become cells of their own (split again at the next level); runs of
// consecutive smaller octants (in Morton order) are merged into one leaf
// while the run holds at most n_split particles, so leaves stay near the
// size of one wave.  Merging is allowed only when the parent already meets
// the extent / smallest-H bound, so a merged leaf never needs a split.
// Writes (first octant, particle begin, count) per child; returns the number
// of children.
__device__ inline int child_groups(const int* bnd, int n_split, bool allow_merge, int* gq, int* gb, int* gc)
{
    int n = 0, open = -1;
    for (int q = 0; q < 8; q++) {
        const int c = bnd[q + 1] - bnd[q];
        if (c == 0) continue;
        if (c > n_split || !allow_merge) {
            open = -1;
            gq[n] = q; gb[n] = bnd[q]; gc[n] = c;
            n++;
            continue;
        }
        if (open >= 0 && gc[open] + c <= n_split) {
            gc[open] += c;
            continue;
        }
        gq[n] = q; gb[n] = bnd[q]; gc[n] = c;
        open = n;
        n++;
    }
    return n;
}

// Whether a cell with these statistics must be split for precision: its
// extent exceeds h_ratio times its smallest H (FP32 cell-relative
// coordinates keep an absolute error of ~1e-7 of the cell extent).
__device__ inline bool extent_too_large(const Node& nd, double h_ratio)
{
    if (!(h_ratio > 0.0) || nd.count < 2) return false;
    const double ext = fmax(fmax(nd.hi[0] - nd.lo[0], nd.hi[1] - nd.lo[1]), nd.hi[2] - nd.lo[2]);
    return ext > h_ratio * nd.hmin;
}

// Statistics of the cells of one level (bounding box, largest and smallest
// H) and the particle bounds of their octants, from chunks of up to
// STATS_CHUNK particles of one cell, one wave per chunk.  Box corners and H
// are >= 0 (validated), so their doubles order like their bit patterns as
// signed 64-bit integers (and so do the -inf / +inf starting values): the
// chunks meet in 64-bit integer atomics min / max, which give exactly the
// minima and maxima of the doubles.  A -0 (which passes the validation)
// enters as +0: its bit pattern would order below -inf.
#define STATS_CHUNK 1024

__device__ inline long long stats_bits(double v)
{
    return __double_as_longlong(v == 0.0 ? 0.0 : v);
}
__device__ inline void atomic_min_d(double* p, double v)
{
    atomicMin((long long*)p, stats_bits(v));
}
__device__ inline void atomic_max_d(double* p, double v)
{
    atomicMax((long long*)p, stats_bits(v));
}

// Chunks of each cell, and the octant bounds [bnd[0..8]] of each cell set to
// its end (the stats pass writes every bound up to the last octant present).
__global__ __launch_bounds__(256) void k_level_chunks(const Node* __restrict__ nodes, int level_start, int n_level,
                                                      int* nchunk, int* bnd)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_level) return;
    const Node& nd = nodes[level_start + k];
    nchunk[k] = (nd.count + STATS_CHUNK - 1) / STATS_CHUNK;
    for (int q = 0; q < 9; q++) bnd[9 * k + q] = nd.begin + nd.count;
}

__global__ __launch_bounds__(256) void k_chunk_map(const int* __restrict__ nchunk, const int* __restrict__ coff,
                                                   int n_level, int* cmap)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_level) return;
    for (int j = 0; j < nchunk[k]; j++) cmap[coff[k] + j] = k;
}

// One wave per chunk (grid-stride over the n_chunks[0] chunks).  Octant of a
// particle in a cell of level `level`: key bits 3 (D - level - 1) and up; the
// first particle of each octant present sets the bounds from the previous
// octant present (exclusive) to its own (inclusive).
__global__ __launch_bounds__(256) void k_level_stats(Node* nodes, int level_start, int level, const int* __restrict__ coff,
                                                     const int* __restrict__ cmap, const int* __restrict__ n_chunks,
                                                     const uint64_t* __restrict__ keys, const double* __restrict__ x,
                                                     const double* __restrict__ y, const double* __restrict__ z,
                                                     const double* __restrict__ H, int D, int* bnd)
{
    const int lane = threadIdx.x & 63;
    const int T = __builtin_amdgcn_readfirstlane(*n_chunks);
    const int shift = 3 * (D - level - 1);
    for (int q = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)); q < T; q += gridDim.x * 4) {
        const int k = __builtin_amdgcn_readfirstlane(cmap[q]);
        Node* nd = &nodes[level_start + k];
        const int b = nd->begin, c = nd->count;
        const bool octants = level < D && !nd->merged;
        const int i0 = b + (q - coff[k]) * STATS_CHUNK, i1 = min(b + c, i0 + STATS_CHUNK);
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double hm = 0.0, hn = INFINITY;
        for (int i = i0 + lane; i < i1; i += 64) {
            const double p[3] = {x[i], y[i], z[i]}, h = H[i];
            for (int a = 0; a < 3; a++) {
                lo[a] = fmin(lo[a], p[a]);
                hi[a] = fmax(hi[a], p[a]);
            }
            hm = fmax(hm, h);
            hn = fmin(hn, h);
            if (octants) {
                const int o = (int)((keys[i] >> shift) & 7);
                const int op = i > b ? (int)((keys[i - 1] >> shift) & 7) : -1;
                for (int r = op + 1; r <= o; r++) bnd[9 * k + r] = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            for (int a = 0; a < 3; a++) {
                lo[a] = fmin(lo[a], __shfl_xor(lo[a], off));
                hi[a] = fmax(hi[a], __shfl_xor(hi[a], off));
            }
            hm = fmax(hm, __shfl_xor(hm, off));
            hn = fmin(hn, __shfl_xor(hn, off));
        }
        if (lane == 0) {
            for (int a = 0; a < 3; a++) {
                atomic_min_d(&nd->lo[a], lo[a]);
                atomic_max_d(&nd->hi[a], hi[a]);
            }
            atomic_max_d(&nd->hmax, hm);
            atomic_min_d(&nd->hmin, hn);
        }
    }
}

// Whether each cell of the level is split and into how many children.  One
// thread per cell.
__global__ __launch_bounds__(256) void k_level_split(Node* nodes, int level_start, int n_level, int D, int n_split,
                                                     double h_ratio, const int* __restrict__ bnd, int* nchild)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_level) return;
    Node* nd = &nodes[level_start + k];
    const bool wide = extent_too_large(*nd, h_ratio);
    const bool split = !nd->merged && nd->level < D && (nd->count > n_split || wide);
    int nc = 0;
    if (split) {
        int bq[9], gq[8], gb[8], gc[8];
        for (int q = 0; q < 9; q++) bq[q] = bnd[9 * k + q];
        nc = child_groups(bq, n_split, !wide, gq, gb, gc);
    }
    nchild[k] = nc;
    nd->n_child = nc;
    nd->first_child = -1;
}

// The children of the split cells, at the scanned offsets.  One thread per
// cell.
__global__ __launch_bounds__(256) void k_emit_children(Node* nodes, int level_start, int n_level, const int* __restrict__ coff,
                                                       int child_base, int D, int n_split, double h_ratio,
                                                       const int* __restrict__ bnd)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_level) return;
    Node* nd = &nodes[level_start + k];
    if (nd->n_child == 0) return;
    const uint64_t step = 1ull << (3 * (D - nd->level - 1));
    int bq[9], gq[8], gb[8], gc[8];
    for (int q = 0; q < 9; q++) bq[q] = bnd[9 * k + q];
    const int ng = child_groups(bq, n_split, !extent_too_large(*nd, h_ratio), gq, gb, gc);
    const int out = child_base + coff[k];
    nd->first_child = out;
    for (int g = 0; g < ng; g++) {
        const int q = gq[g];
        Node ch;
        ch.key_lo = nd->key_lo + step * q;
        ch.begin = gb[g];
        ch.count = gc[g];
        ch.first_child = -1;
        ch.n_child = 0;
        ch.level = nd->level + 1;
        ch.domain = nd->domain;
        ch.leaf = -1;
        ch.top = nd->top;
        const int o[3] = {(q >> 2) & 1, (q >> 1) & 1, q & 1};
        for (int a = 0; a < 3; a++) {
            ch.c_sz[a] = 0.5 * nd->c_sz[a];
            ch.c_lo[a] = nd->c_lo[a] + o[a] * ch.c_sz[a];
            ch.lo[a] = INFINITY;
            ch.hi[a] = -INFINITY;
        }
        ch.hmax = 0.0;
        ch.hmin = INFINITY;
        ch.merged = (q + 1 < 8 && gb[g] + gc[g] > bq[q + 1]) ? 1 : 0;
        ch.pad = 0;
        nodes[out + g] = ch;
    }
}

__global__ __launch_bounds__(256) void k_mark_leaves(const Node* __restrict__ nodes, int n_nodes, int* leafmark)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    const Node& nd = nodes[k];
    if (nd.n_child == 0 && nd.count > 0) leafmark[nd.begin] = 1;
}

__global__ __launch_bounds__(256) void k_leaf_fill(Node* nodes, int n_nodes, const int* __restrict__ leafscan,
                                                   int* leaf_node, int* l_begin, int* l_count, double* l_origin,
                                                   double* l_lo, double* l_hi, double* l_hlist, int* l_dom, int* l_top,
                                                   double skin_abs, int* max_leaf)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    Node& nd = nodes[k];
    if (!(nd.n_child == 0 && nd.count > 0)) {
        nd.leaf = -1;
        return;
    }
    if (nd.count > 64) atomicMax(max_leaf, nd.count);
    const int id = leafscan[nd.begin];
    nd.leaf = id;
    leaf_node[id] = k;
    l_begin[id] = nd.begin;
    l_count[id] = nd.count;
    for (int a = 0; a < 3; a++) {
        l_lo[3 * id + a] = nd.lo[a];
        l_hi[3 * id + a] = nd.hi[a];
        l_origin[3 * id + a] = 0.5 * (nd.lo[a] + nd.hi[a]);
    }
    l_hlist[id] = nd.hmax * (1.0 + SPH_LIST_SKIN) + skin_abs;
    l_dom[id] = nd.domain;
    l_top[id] = nd.top;
}

// Cell-relative coordinates (and masses) of every particle in its leaf.
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_pos(int n_leaves, const int* __restrict__ l_begin,
                                                  const int* __restrict__ l_count, const double* __restrict__ l_origin,
                                                  const double* __restrict__ x, const double* __restrict__ y,
                                                  const double* __restrict__ z, const double* __restrict__ m,
                                                  const double* __restrict__ H, typename vec4<T>::type* pos4, T* hf)
{
    const int A = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (A >= n_leaves) return;
    const int lane = threadIdx.x & 63;
    const int b = l_begin[A], c = l_count[A];
    const double ox = l_origin[3 * A], oy = l_origin[3 * A + 1], oz = l_origin[3 * A + 2];
    for (int p = b + lane; p < b + c; p += 64) {
        typename vec4<T>::type v;
        v.x = (T)(x[p] - ox);
        v.y = (T)(y[p] - oy);
        v.z = (T)(z[p] - oz);
        v.w = (T)m[p];
        pos4[p] = v;
        hf[p] = (T)H[p];
    }
}

// Refresh of the cell-relative coordinates after a drift without a rebuild:
// the nearest periodic image of each particle relative to its leaf's
// origin, and the test that the leaf's largest H plus the displacement
// margin still lies inside the radius its list was built for.  In the FP32
// modes (ext_ratio > 0) a leaf that could still be split and whose extent
// plus the motion exceeds ext_ratio times its smallest H also asks for a
// rebuild (the extent rule of the build, with the hysteresis of the check
// after a density call).
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_refresh(int n_leaves, const int* __restrict__ l_begin,
                                                      const int* __restrict__ l_count, const double* __restrict__ l_origin,
                                                      const double* __restrict__ l_hlist, const int* __restrict__ l_dom,
                                                      const DomainInfo* __restrict__ di, const double* __restrict__ x,
                                                      const double* __restrict__ y, const double* __restrict__ z,
                                                      const double* __restrict__ m, const double* __restrict__ H,
                                                      const double* __restrict__ margin, typename vec4<T>::type* pos4,
                                                      T* hf, int* flags, const double* __restrict__ l_lo,
                                                      const double* __restrict__ l_hi, const int* __restrict__ leaf_node,
                                                      const Node* __restrict__ nodes, int max_level, double ext_ratio)
{
    const int A = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (A >= n_leaves) return;
    const int lane = threadIdx.x & 63;
    const int b = l_begin[A], c = l_count[A];
    const double o[3] = {l_origin[3 * A], l_origin[3 * A + 1], l_origin[3 * A + 2]};
    const DomainInfo& I = di[l_dom[A]];
    double hm = 0.0, hn = INFINITY;
    for (int p = b + lane; p < b + c; p += 64) {
        const double q[3] = {x[p], y[p], z[p]};
        T r[3];
        for (int a = 0; a < 3; a++) {
            double d = q[a] - o[a];
            if (d > 0.5 * I.L[a]) d -= I.L[a];
            else if (d < -0.5 * I.L[a]) d += I.L[a];
            r[a] = (T)d;
        }
        typename vec4<T>::type v;
        v.x = r[0];
        v.y = r[1];
        v.z = r[2];
        v.w = (T)m[p];
        pos4[p] = v;
        const double h = H[p];
        hf[p] = (T)h;
        hm = fmax(hm, h);
        hn = fmin(hn, h);
    }
    for (int off = 32; off > 0; off >>= 1) {
        hm = fmax(hm, __shfl_xor(hm, off));
        hn = fmin(hn, __shfl_xor(hn, off));
    }
    bool stale = !(hm + *margin < l_hlist[A]);
    if (ext_ratio > 0.0 && c >= 2 && nodes[leaf_node[A]].level < max_level) {
        const double ext = fmax(fmax(l_hi[3 * A] - l_lo[3 * A], l_hi[3 * A + 1] - l_lo[3 * A + 1]),
                                l_hi[3 * A + 2] - l_lo[3 * A + 2]) + *margin;
        stale = stale || ext > ext_ratio * hn;
    }
    if (lane == 0 && stale) atomicOr(flags, FLAG_STALE);
}

// ---------------------------------------------------------------------------
// Neighbour-cell lists (gather form).  Leaf A's list holds every leaf B (with
// periodic image) whose bounding box lies closer to A's than h_A, the radius
// A's list is built for (largest H in A plus a skin): these are the cells the
// density sum of eq. (rho) over r < H_i needs.  The symmetric force range
// r < max(H_i, H_j) of eq. (dvdt) is covered by the union of A's and B's
// lists; each unordered pair of cells is evaluated once by a fixed owner
// (see force_owner).  With the gather-form force the lists are symmetric:
// A's list also holds every B whose own radius h_B reaches A's box, so that
// each particle finds all its pairs r < max(H_i, H_j) in its own cell's list.
// Found by descending the octree from the 27 top cells around A's top cell,
// pruning cells whose box lies farther away than h_A (and than the largest
// list radius below them, for symmetric lists).
// ---------------------------------------------------------------------------

__device__ inline double box_dist(const double* alo, const double* ahi, const double* blo, const double* bhi,
                                  const double* s)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; a++) {
        const double lo = blo[a] + s[a], hi = bhi[a] + s[a];
        double g = 0.0;
        if (lo > ahi[a]) g = lo - ahi[a];
        else if (alo[a] > hi) g = alo[a] - hi;
        d2 += g * g;
    }
    return sqrt(d2);
}

__constant__ float c_dirs[SPH_NDIR][3] = {
    {1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f},
    {0.70710678f, 0.70710678f, 0.f}, {0.70710678f, -0.70710678f, 0.f},
    {0.70710678f, 0.f, 0.70710678f}, {0.70710678f, 0.f, -0.70710678f},
    {0.f, 0.70710678f, 0.70710678f}, {0.f, 0.70710678f, -0.70710678f},
    {0.57735027f, 0.57735027f, 0.57735027f}, {0.57735027f, 0.57735027f, -0.57735027f},
    {0.57735027f, -0.57735027f, 0.57735027f}, {0.57735027f, -0.57735027f, -0.57735027f}};

__global__ __launch_bounds__(256) void k_wnodes(const Node* __restrict__ nodes, int n_nodes, double skin_abs,
                                                WNode* __restrict__ w)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    const Node& nd = nodes[k];
    WNode o;
    for (int a = 0; a < 3; a++) {
        o.lo[a] = __double2float_rd(nd.lo[a]);
        o.hi[a] = __double2float_ru(nd.hi[a]);
    }
    o.first_child = nd.n_child > 0 ? nd.first_child : -1;
    o.next = -1;
    o.count = nd.count;
    o.leaf = nd.leaf;
    // float bound of the subtree's list radii (as k_node_hmax sets it)
    o.hl = __double2float_ru((nd.hmax * (1.0 + SPH_LIST_SKIN) + skin_abs) * (1.0 + 1e-6));
    o.pad = nd.n_child;
    w[k] = o;
}

// Escape links, one level at a time from the top: a child's next node is its
// next sibling, the last child inherits its parent's next node.
__global__ __launch_bounds__(256) void k_wnext(const Node* __restrict__ nodes, int level_start, int n_level,
                                               WNode* __restrict__ w)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_level) return;
    const int p = level_start + k;
    const Node& nd = nodes[p];
    if (nd.n_child == 0) return;
    const int pn = w[p].next;
    for (int q = 0; q < nd.n_child; q++) w[nd.first_child + q].next = (q + 1 < nd.n_child) ? nd.first_child + q + 1 : pn;
}

__device__ inline float box_dist_f(const float* alo, const float* ahi, const float* blo, const float* bhi,
                                   const float* s)
{
    float d2 = 0.f;
    for (int a = 0; a < 3; a++) {
        const float lo = blo[a] + s[a], hi = bhi[a] + s[a];
        float g = 0.f;
        if (lo > ahi[a]) g = lo - ahi[a];
        else if (alo[a] > hi) g = alo[a] - hi;
        d2 += g * g;
    }
    return sqrtf(d2);
}

// Sort direction of a listed pair: the one of the 13 most aligned with the
// offset between the box centres (B's image).
__device__ inline int walk_dir(const double* alo, const double* ahi, const double* blo, const double* bhi,
                               const double* sv)
{
    float cv[3];
    for (int a = 0; a < 3; a++) cv[a] = (float)(0.5 * (blo[a] + bhi[a]) + sv[a] - 0.5 * (alo[a] + ahi[a]));
    float bv = -1.f;
    int best = 0;
    for (int q = 0; q < SPH_NDIR; q++) {
        const float v = fabsf(cv[0] * c_dirs[q][0] + cv[1] * c_dirs[q][1] + cv[2] * c_dirs[q][2]);
        if (v > bv) { bv = v; best = q; }
    }
    return best;
}

// Exact distance between the leaf boxes of A and B's image (shift sv), in
// the canonical order, so that both lists of a pair hold the same value.
__device__ inline double walk_pair_dist(int A, int B, const double* alo, const double* ahi, const double* blo,
                                        const double* bhi, const double* sv)
{
    const bool fwd = A <= B;
    double plo[3], phi[3], qlo[3], qhi[3], s[3];
    for (int a = 0; a < 3; a++) {
        plo[a] = fwd ? alo[a] : blo[a];
        phi[a] = fwd ? ahi[a] : bhi[a];
        qlo[a] = fwd ? blo[a] : alo[a];
        qhi[a] = fwd ? bhi[a] : ahi[a];
        s[a] = fwd ? sv[a] : -sv[a];
    }
    return box_dist(plo, phi, qlo, qhi, s);
}

// Output of one leaf's walk.  MODE 1: at the scanned offsets; MODE 2:
// the first `len` entries into the leaf's slot, the rest into 64-entry
// chunks of `ovf` taken one at a time (link: [head of each leaf's chain |
// state of each leaf | next chunk]); a leaf that finds no free chunk keeps
// counting and is walked again at the scanned offsets.
struct WalkSink {
    size_t base;
    int len, out, cnt, last;
    bool failed;
};

template <int MODE>
__device__ inline void walk_put(WalkSink& s, int A, const ListEntry& e, ListEntry* list, ListEntry* ovf, int* link,
                                int* next, int* flags, int ovf_chunks)
{
    ListEntry* dst = nullptr;
    if (s.out < s.len) {
        dst = list + s.base + s.out;
    } else if (MODE == 2 && !s.failed) {
        const int k = s.out - s.len;
        if ((k & 63) == 0) {
            const int ch = atomicAdd(flags + FI_WOVF, 1);
            if (ch >= ovf_chunks) {
                s.failed = true;
            } else {
                if (s.last < 0) link[A] = ch;
                else next[s.last] = ch;
                next[ch] = -1;
                s.last = ch;
            }
        }
        if (!s.failed) dst = ovf + (size_t)s.last * 64 + (k & 63);
    }
    if (dst) *dst = e;
    else if (MODE == 1) atomicOr(flags, FLAG_INVALID);
    s.out++;
}

// Closing bookkeeping of a MODE 2 walk of leaf A.
__device__ inline void walk_close(const WalkSink& s, int A, int n_leaves, int list_cap, int* counts, int* link, int* flags)
{
    counts[A] = s.cnt;
    if (s.cnt > list_cap) atomicMax(flags + FI_MAXLIST, s.cnt);
    if (s.last < 0) link[A] = -1;
    link[n_leaves + A] = s.failed ? 1 : 0;
    if (s.failed) atomicAdd(flags + FI_WINC, 1);
}

// One thread per leaf A.  MODE 0: count the entries of each leaf; 1: write
// them at the scanned offsets l_off (with `link`, only the leaves it marks
// incomplete); 2: write into the slot and overflow chunks and count them
// (WalkSink).
template <int MODE>
__global__ __launch_bounds__(128) void k_walk(int n_leaves, const int* __restrict__ leaf_node, const WNode* __restrict__ wn,
                                              const double* __restrict__ l_lo, const double* __restrict__ l_hi,
                                              const int* __restrict__ l_dom, const int* __restrict__ l_top,
                                              const DomainInfo* __restrict__ di, const double* __restrict__ l_hlist,
                                              int* counts, const int* __restrict__ l_off, ListEntry* __restrict__ list,
                                              int list_cap, int with_dir, int sym, int* flags, ListEntry* ovf,
                                              int* link, int ovf_chunks)
{
    const int A = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (A >= n_leaves) return;
    if (MODE == 1 && link && !link[n_leaves + A]) return;
    int* next = link ? link + 2 * (size_t)n_leaves : nullptr;
    const DomainInfo& I = di[l_dom[A]];
    const int loc = l_top[A] - I.top_offset;
    const int tc[3] = {loc / (I.n_top[2] * I.n_top[1]), (loc / I.n_top[2]) % I.n_top[1], loc % I.n_top[2]};
    const double hA = l_hlist[A];
    // conservative float pruning radius: the float boxes are rounded outward;
    // the absolute term covers the rounding of box + periodic shift in float
    const float slack = (float)(1e-6 * fmax(fmax(I.L[0], I.L[1]), I.L[2]));
    const float prune = (float)(hA * (1.0 + 1e-5)) + slack;
    const WNode& WA = wn[leaf_node[A]];
    const double alo[3] = {l_lo[3 * A], l_lo[3 * A + 1], l_lo[3 * A + 2]};
    const double ahi[3] = {l_hi[3 * A], l_hi[3 * A + 1], l_hi[3 * A + 2]};
    constexpr bool FILL = MODE != 0;
    WalkSink s;
    s.base = MODE == 1 ? (size_t)l_off[A] : (MODE >= 2 ? (size_t)A * list_cap : 0);
    s.len = MODE == 1 ? l_off[A + 1] - l_off[A] : (MODE >= 2 ? list_cap : 0);
    s.out = 0;
    s.cnt = 0;
    s.last = -1;
    s.failed = false;
    for (int sx = -1; sx <= 1; sx++)
    for (int sy = -1; sy <= 1; sy++)
    for (int sz = -1; sz <= 1; sz++) {
        const int o[3] = {sx, sy, sz};
        int nc[3], ps[3];
        double sv[3];
        float svf[3];
        for (int a = 0; a < 3; a++) {
            nc[a] = tc[a] + o[a];
            ps[a] = 0;
            if (nc[a] < 0) { nc[a] += I.n_top[a]; ps[a] = -1; }
            else if (nc[a] >= I.n_top[a]) { nc[a] -= I.n_top[a]; ps[a] = 1; }
            sv[a] = ps[a] * I.L[a];
            svf[a] = (float)sv[a];
        }
        const int code_shift = shift_index(ps[0], ps[1], ps[2]);
        // depth-first over the neighbour top cell without a stack: descend to
        // the first child, or skip the subtree through its escape link
        int k = I.top_offset + (nc[0] * I.n_top[1] + nc[1]) * I.n_top[2] + nc[2];
        while (k >= 0) {
            const WNode nd = wn[k];
            // symmetric lists also take every leaf whose own radius reaches A
            if (nd.count == 0 ||
                box_dist_f(WA.lo, WA.hi, nd.lo, nd.hi, svf) > (sym ? fmaxf(prune, nd.hl * 1.00001f + slack) : prune)) {
                k = nd.next;
                continue;
            }
            if (nd.first_child >= 0) {
                k = nd.first_child;
                continue;
            }
            k = nd.next;
            const int B = nd.leaf;
            const double blo[3] = {l_lo[3 * B], l_lo[3 * B + 1], l_lo[3 * B + 2]};
            const double bhi[3] = {l_hi[3 * B], l_hi[3 * B + 1], l_hi[3 * B + 2]};
            const double d = walk_pair_dist(A, B, alo, ahi, blo, bhi, sv);
            if (!(d < (sym ? fmax(hA, l_hlist[B]) : hA))) continue;
            if (FILL) {
                ListEntry e;
                e.B = B;
                e.code = code_shift | ((with_dir ? walk_dir(alo, ahi, blo, bhi, sv) : 0) << 8);
                e.dist = d;
                walk_put<MODE>(s, A, e, list, ovf, link, next, flags, ovf_chunks);
            }
            s.cnt++;
        }
    }
    if (MODE == 0) counts[A] = s.cnt;
    if (MODE >= 2) walk_close(s, A, n_leaves, list_cap, counts, link, flags);
}

// Stack entries per wave of the wave walk, and the room it keeps free: a
// round that pops p cells pushes at most 8p children, so rounds pop no more
// than keeps 7p below the reserve; one cell at a time (a plain depth-first
// descent) grows the stack by at most 7 per level below the top grid.
#define WALK_STACK 1024
#define WALK_RESERVE (7 * (SPH_MAX_DEPTH + 1))
static_assert(WALK_STACK - WALK_RESERVE >= 8 * 27, "the first round's children must fit");

__device__ inline void walk_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Float cell test of the wave walk, as a squared distance with a relative
// margin of 1e-5: it never rejects a cell that box_dist_f(...) <= r accepts
// (the margin is far above the rounding of the square and of r^2), so the
// wave walk reaches every cell the one-leaf walk reaches.
__device__ inline bool walk_near_f(const float* alo, const float* ahi, const float* blo, const float* bhi,
                                   const float* s, float r)
{
    float d2 = 0.f;
    for (int a = 0; a < 3; a++) {
        const float g = fmaxf(fmaxf((blo[a] + s[a]) - ahi[a], alo[a] - (bhi[a] + s[a])), 0.f);
        d2 = fmaf(g, g, d2);
    }
    return d2 <= r * r * 1.00001f;
}

// The MODE 2 walk of one leaf A by a whole wave: the descent of k_walk from
// the 27 top cells around A's top cell, up to 64 cells per round (one per
// lane) popped from a stack in LDS, the exact test of each leaf cell reached
// in its own lane, and the entries of a round appended in lane order (the
// same order on every run).  Each leaf gets the entries of k_walk<2>: the
// float test is looser, and every entry passes the same exact test (which
// implies the float test).  A round's entries go to the slot, then to
// 64-entry chunks of the pool (at most two new ones per round).  One wave
// per leaf, four per workgroup, eight waves per SIMD (64 VGPRs, no spills;
// the walk waits on its loads).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_walk_wave(
    int n_leaves, const int* __restrict__ leaf_node, const WNode* __restrict__ wn, const double* __restrict__ l_lo,
    const double* __restrict__ l_hi, const int* __restrict__ l_dom, const int* __restrict__ l_top,
    const DomainInfo* __restrict__ di, const double* __restrict__ l_hlist, int* counts, ListEntry* __restrict__ list,
    int list_cap, int with_dir, int sym, int* flags, ListEntry* ovf, int* link, int ovf_chunks)
{
    __shared__ uint32_t stk[4][WALK_STACK];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int A = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * 4 + w);
    if (A >= n_leaves) return;
    int* next = link + 2 * (size_t)n_leaves;
    const DomainInfo& I = di[l_dom[A]];
    const int nt[3] = {I.n_top[0], I.n_top[1], I.n_top[2]};
    const double L[3] = {I.L[0], I.L[1], I.L[2]};
    const float Lf[3] = {(float)L[0], (float)L[1], (float)L[2]};
    const int loc = l_top[A] - I.top_offset;
    const int tc[3] = {loc / (nt[2] * nt[1]), (loc / nt[2]) % nt[1], loc % nt[2]};
    const double hA = l_hlist[A];
    // conservative float radius, as in k_walk
    const float slack = (float)(1e-6 * fmax(fmax(L[0], L[1]), L[2]));
    const float prune = (float)(hA * (1.0 + 1e-5)) + slack;
    const WNode& WA = wn[leaf_node[A]];
    const float wlo[3] = {WA.lo[0], WA.lo[1], WA.lo[2]}, whi[3] = {WA.hi[0], WA.hi[1], WA.hi[2]};
    const double alo[3] = {l_lo[3 * A], l_lo[3 * A + 1], l_lo[3 * A + 2]};
    const double ahi[3] = {l_hi[3 * A], l_hi[3 * A + 1], l_hi[3 * A + 2]};
    // output state (wave-uniform): entries so far, chunks taken, the last one
    int out = 0, n_chunks = 0, last = -1;
    bool failed = false;
    int size = 0;
    bool first_round = true;
    while (first_round || size > 0) {
        int node = -1, sc = 0;
        if (first_round) {
            // the 27 top cells around A's and their periodic images
            if (lane < 27) {
                const int o[3] = {lane / 9 - 1, (lane / 3) % 3 - 1, lane % 3 - 1};
                int cc[3], ps[3];
                for (int a = 0; a < 3; a++) {
                    cc[a] = tc[a] + o[a];
                    ps[a] = cc[a] < 0 ? -1 : (cc[a] >= nt[a] ? 1 : 0);
                    cc[a] -= ps[a] * nt[a];
                }
                node = I.top_offset + (cc[0] * nt[1] + cc[1]) * nt[2] + cc[2];
                sc = shift_index(ps[0], ps[1], ps[2]);
            }
            first_round = false;
        } else {
            int p = min(min(64, size), (WALK_STACK - WALK_RESERVE - size) / 7);
            if (p < 1) p = 1;
            size -= p;
            if (lane < p) {
                const uint32_t e = stk[w][size + lane];
                node = (int)(e >> 5);
                sc = (int)(e & 31);
            }
        }
        const int ps[3] = {sc / 9 - 1, (sc / 3) % 3 - 1, sc % 3 - 1};
        int first = -1, n_child = 0, B = -1;
        if (node >= 0) {
            const WNode nd = wn[node];
            float svf[3];
            for (int a = 0; a < 3; a++) svf[a] = ps[a] < 0 ? -Lf[a] : (ps[a] > 0 ? Lf[a] : 0.f);
            if (nd.count != 0 &&
                walk_near_f(wlo, whi, nd.lo, nd.hi, svf, sym ? fmaxf(prune, nd.hl * 1.00001f + slack) : prune)) {
                if (nd.first_child >= 0) {
                    first = nd.first_child;
                    n_child = nd.pad;
                } else {
                    B = nd.leaf;
                }
            }
        }
        // children go on the stack in lane order (a wave-wide prefix sum)
        {
            int pre = n_child;
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(pre, off);
                if (lane >= off) pre += t;
            }
            const int total = __builtin_amdgcn_readlane(pre, 63);
            pre -= n_child;
            for (int j = 0; j < n_child; j++) stk[w][size + pre + j] = ((uint32_t)(first + j) << 5) | (uint32_t)sc;
            size += total;
        }
        // exact test of the leaf cells reached, one per lane
        bool hit = false;
        ListEntry en;
        if (B >= 0) {
            double blo[3], bhi[3];
            for (int a = 0; a < 3; a++) {
                blo[a] = l_lo[3 * B + a];
                bhi[a] = l_hi[3 * B + a];
            }
            const double sv[3] = {ps[0] * L[0], ps[1] * L[1], ps[2] * L[2]};
            const double d = walk_pair_dist(A, B, alo, ahi, blo, bhi, sv);
            hit = d < (sym ? fmax(hA, l_hlist[B]) : hA);
            en.B = B;
            en.code = sc | ((with_dir ? walk_dir(alo, ahi, blo, bhi, sv) : 0) << 8);
            en.dist = d;
        }
        const unsigned long long hm = __ballot(hit);
        if (hm) {
            const int k = __popcll(hm);
            const int pos = out + __popcll(hm & ((1ull << lane) - 1ull));
            // ch[0]: chunk jl of the round's first position past the slot (the
            // last chunk taken when that one is partly filled), ch[1]: jl + 1
            const int jl = out > list_cap ? (out - list_cap) >> 6 : 0;
            int ch[2] = {last, -1};
            if (!failed && out + k > list_cap) {
                const int jh = (out + k - 1 - list_cap) >> 6;
                for (int j = n_chunks; j <= jh; j++) {
                    int c = 0;
                    if (lane == 0) c = atomicAdd(flags + FI_WOVF, 1);
                    c = __builtin_amdgcn_readfirstlane(c);
                    if (c >= ovf_chunks) {
                        failed = true;
                        break;
                    }
                    if (lane == 0) {
                        if (last < 0) link[A] = c;
                        else next[last] = c;
                        next[c] = -1;
                    }
                    last = c;
                    n_chunks = j + 1;
                    ch[j - jl] = c;
                }
            }
            if (hit) {
                ListEntry* dst = nullptr;
                if (pos < list_cap) {
                    dst = list + (size_t)A * list_cap + pos;
                } else {
                    const int j = (pos - list_cap) >> 6;
                    if (j < n_chunks) dst = ovf + (size_t)ch[j - jl] * 64 + ((pos - list_cap) & 63);
                }
                if (dst) *dst = en;
            }
            out += k;
        }
        // the next round reads the stack this one wrote
        walk_wave_sync();
    }
    if (lane == 0) {
        counts[A] = out;
        if (out > list_cap) atomicMax(flags + FI_MAXLIST, out);
        if (last < 0) link[A] = -1;
        link[n_leaves + A] = failed ? 1 : 0;
        if (failed) atomicAdd(flags + FI_WINC, 1);
    }
}

// Move the entries of the one-pass walk from the per-leaf slots and their
// overflow chains to the scanned offsets (incomplete leaves are walked
// again).  One wave per leaf.
__global__ __launch_bounds__(256) void k_list_compact(int n_leaves, int cap, const ListEntry* __restrict__ scratch,
                                                      const ListEntry* __restrict__ ovf, const int* __restrict__ link,
                                                      const int* __restrict__ l_off, ListEntry* __restrict__ list)
{
    const int A = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (A >= n_leaves) return;
    if (link[n_leaves + A]) return;
    const int lane = threadIdx.x & 63;
    const int o = l_off[A], n = l_off[A + 1] - o;
    const int ns = min(n, cap);
    for (int e = lane; e < ns; e += 64) list[o + e] = scratch[(size_t)A * cap + e];
    const int* next = link + 2 * (size_t)n_leaves;
    int ch = __builtin_amdgcn_readfirstlane(link[A]);
    for (int b = ns; b < n && ch >= 0; b += 64) {
        if (b + lane < n) list[o + b + lane] = ovf[(size_t)ch * 64 + lane];
        ch = __builtin_amdgcn_readfirstlane(next[ch]);
    }
}

// Largest H per cell, bottom-up over one level (leaves from particles,
// internal cells from children).  One wave per cell.
__global__ __launch_bounds__(256) void k_node_hmax(Node* nodes, int level_start, int n_level, const double* __restrict__ H,
                                                   double* l_hlist, double skin_abs, WNode* wn)
{
    const int k = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (k >= n_level) return;
    const int lane = threadIdx.x & 63;
    Node& nd = nodes[level_start + k];
    double hm = 0.0;
    if (nd.n_child == 0) {
        for (int p = nd.begin + lane; p < nd.begin + nd.count; p += 64) hm = fmax(hm, H[p]);
    } else if (lane < nd.n_child) {
        hm = nodes[nd.first_child + lane].hmax;
    }
    for (int off = 32; off > 0; off >>= 1) hm = fmax(hm, __shfl_xor(hm, off));
    if (lane == 0) {
        nd.hmax = hm;
        if (nd.leaf >= 0 && l_hlist) l_hlist[nd.leaf] = hm * (1.0 + SPH_LIST_SKIN) + skin_abs;
        // float bound of the subtree's list radii for the symmetric walk
        if (wn) wn[level_start + k].hl = __double2float_ru((hm * (1.0 + SPH_LIST_SKIN) + skin_abs) * (1.0 + 1e-6));
    }
}

// ---------------------------------------------------------------------------
// Sort stage: per leaf and direction, projections of the cell-relative
// positions sorted ascending (bitonic network across the 64 lanes).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sort_cells(int n_leaves, int64_t n, const int* __restrict__ l_begin,
                                                    const int* __restrict__ l_count,
                                                    const typename vec4<T>::type* __restrict__ pos4,
                                                    float* __restrict__ skey, uint16_t* __restrict__ sidx, int* l_sorted)
{
    const int A = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (A >= n_leaves) return;
    const int lane = threadIdx.x & 63;
    const int b = l_begin[A], c = l_count[A];
    if (c > 64) {
        if (lane == 0) l_sorted[A] = 0;
        return;
    }
    T px = 0, py = 0, pz = 0;
    if (lane < c) {
        const typename vec4<T>::type p = pos4[b + lane];
        px = p.x; py = p.y; pz = p.z;
    }
    for (int d = 0; d < SPH_NDIR; d++) {
        double u[3];
        sph_dir(d, u);
        float key = (lane < c) ? (float)((double)px * u[0] + (double)py * u[1] + (double)pz * u[2]) : INFINITY;
        int idx = lane;
        for (int k = 2; k <= 64; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                const float pk = __shfl_xor(key, j);
                const int pi = __shfl_xor(idx, j);
                const bool up = (lane & k) == 0;
                const bool lower = (lane & j) == 0;
                const bool want_min = (lower == up);
                const bool take = want_min ? (pk < key || (pk == key && pi < idx)) : (pk > key || (pk == key && pi > idx));
                if (take) {
                    key = pk;
                    idx = pi;
                }
            }
        }
        if (lane < c) {
            skey[(int64_t)d * n + b + lane] = key;
            sidx[(int64_t)d * n + b + lane] = (uint16_t)idx;
        }
    }
    if (lane == 0) l_sorted[A] = 1;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

static sph_status read_int(sph_ctx* c, const int* dptr, int* out)
{
    SPH_CHECK_HIP(hipMemcpyAsync(out, dptr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    return SPH_OK;
}

// Permutes the caller's arrays by perm.  x, y, z and H, which the octree
// reads next, on the context's stream; the other arrays, when the context
// has a second stream and side_tmp (8 bytes per particle) is given, on that
// stream, after the sort (an event) and joined back by perm_join before
// their first reader, so that they move while the octree is built.
static sph_status permute_all(sph_ctx* c, const uint32_t* perm, void* side_tmp)
{
    const int64_t n = c->n;
    SPH_TRY(buf_ensure(c->tmp, (size_t)n * 8));
    // rho, drho_dH, omega and P follow their particles unless the caller's
    // next stages rewrite them before reading (the build inside a step)
    const bool dens_out = !c->dens_outputs_dead;
    double* geo[] = {c->P.x, c->P.y, c->P.z, c->P.H};
    double* rest[] = {c->P.vx, c->P.vy, c->P.vz, c->P.u, c->P.m,
                      dens_out ? c->P.rho : nullptr, dens_out ? c->P.drho_dH : nullptr,
                      dens_out ? c->P.omega : nullptr, dens_out ? c->P.P : nullptr,
                      c->P.ax, c->P.ay, c->P.az, c->P.dudt};
    const int nb4 = blocks_for((n + 3) / 4, 256);
    const bool split = c->side && side_tmp;
    hipStream_t s2 = split ? c->side : c->stream;
    void* t2 = split ? side_tmp : c->tmp.p;
    if (split) {
        SPH_CHECK_HIP(hipEventRecord(c->side_ev[0], c->stream));
        SPH_CHECK_HIP(hipStreamWaitEvent(c->side, c->side_ev[0], 0));
        c->side_pending = true;
    }
    // gather into tmp, then back (the caller's arrays are 8-byte aligned:
    // the vector copy needs 16)
    auto permute8 = [&](void* a, bool is_id, hipStream_t st, void* tmp) -> sph_status {
        if (is_id) k_gather<int64_t><<<nb4, 256, 0, st>>>(n, perm, (const int64_t*)a, (int64_t*)tmp);
        else k_gather<double><<<nb4, 256, 0, st>>>(n, perm, (const double*)a, (double*)tmp);
        SPH_CHECK_LAUNCH();
        if (((uintptr_t)a & 15) == 0) {
            k_copy8<<<nb4, 256, 0, st>>>(n, (const uint64_t*)tmp, (uint64_t*)a);
            SPH_CHECK_LAUNCH();
        } else {
            SPH_CHECK_HIP(hipMemcpyAsync(a, tmp, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
        }
        return SPH_OK;
    };
    for (double* a : rest)
        if (a) SPH_TRY(permute8(a, false, s2, t2));
    if (c->P.id) SPH_TRY(permute8(c->P.id, true, s2, t2));
    if (c->P.domain) {
        k_gather<int32_t><<<nb4, 256, 0, s2>>>(n, perm, c->P.domain, (int32_t*)t2);
        SPH_CHECK_LAUNCH();
        SPH_CHECK_HIP(hipMemcpyAsync(c->P.domain, t2, (size_t)n * 4, hipMemcpyDeviceToDevice, s2));
    }
    if (split) SPH_CHECK_HIP(hipEventRecord(c->side_ev[1], c->side));
    for (double* a : geo)
        if (a) SPH_TRY(permute8(a, false, c->stream, c->tmp.p));
    if (c->mlp_pending) {
        // predictor features and previous H of this step follow their particles
        k_gather<double><<<nb4, 256, 0, c->stream>>>(n, perm, (const double*)c->mlp_hprev.p, (double*)c->tmp.p);
        SPH_CHECK_LAUNCH();
        SPH_CHECK_HIP(hipMemcpyAsync(c->mlp_hprev.p, c->tmp.p, (size_t)n * 8, hipMemcpyDeviceToDevice, c->stream));
        SPH_TRY(buf_ensure(c->tmp, (size_t)n * sizeof(float4) * 2));
        k_gather<FeatRow><<<nb4, 256, 0, c->stream>>>(n, perm, (const FeatRow*)c->mlp_X.p, (FeatRow*)c->tmp.p);
        SPH_CHECK_LAUNCH();
        SPH_CHECK_HIP(hipMemcpyAsync(c->mlp_X.p, c->tmp.p, (size_t)n * sizeof(FeatRow), hipMemcpyDeviceToDevice,
                                     c->stream));
    }
    return SPH_OK;
}

// The context's stream waits for the arrays permuted on the second stream.
static void perm_join(sph_ctx* c)
{
    if (!c->side_pending) return;
    (void)hipStreamWaitEvent(c->stream, c->side_ev[1], 0);
    c->side_pending = false;
}

// Unordered pair tasks of the neighbour-cell lists: the entries a leaf owns.
// Symmetric lists (gather-form force) hold every pair in both leaves' lists,
// so the entry with B > A owns it; one-sided lists (pairs form) hold B in A's
// list when B is within A's radius, so A also owns the entries whose B does
// not reach back to A.  A statistic only, counted when it is read.
__global__ __launch_bounds__(256) void k_pair_tasks(int n_leaves, const int* __restrict__ l_off,
                                                    const ListEntry* __restrict__ list,
                                                    const double* __restrict__ l_hlist, int sym,
                                                    unsigned long long* n_owned)
{
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long own = 0;
    if (A < n_leaves)
        for (int e = l_off[A]; e < l_off[A + 1]; e++) {
            const ListEntry E = list[e];
            if (E.B != A && (E.B > A || (!sym && !(E.dist < l_hlist[E.B])))) own++;
        }
    for (int off = 32; off > 0; off >>= 1) own += __shfl_xor(own, off);
    if ((threadIdx.x & 63) == 0 && own) atomicAdd(n_owned, own);
}

sph_status count_pair_tasks(sph_ctx* c)
{
    const int nL = c->n_leaves;
    unsigned long long* npair = (unsigned long long*)c->counters.p + CNT_NPAIR;
    SPH_CHECK_HIP(hipMemsetAsync(npair, 0, 8, c->stream));
    if (nL <= 0) return SPH_OK;
    k_pair_tasks<<<blocks_for(nL, 256), 256, 0, c->stream>>>(nL, (const int*)c->l_off.p, (const ListEntry*)c->list.p,
                                                           (const double*)c->l_hlist.p,
                                                           c->prm.force_mode == SPH_FORCE_GATHER ? 1 : 0, npair);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

// Per-box range [begin, end) of the Morton-ordered particles.
__global__ void k_domain_ranges(int ndom, const DomainInfo* __restrict__ di, const uint64_t* __restrict__ keys, int n,
                                int D, int* ranges)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d > ndom) return;
    if (d == ndom) {
        ranges[d] = n;
        return;
    }
    const uint64_t k = (uint64_t)di[d].top_offset << (3 * D);
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    ranges[d] = lo;
}

sph_status domain_ranges(sph_ctx* c)
{
    const int nd = c->prm.n_domains;
    k_domain_ranges<<<blocks_for(nd + 1, 64), 64, 0, c->stream>>>(nd, (const DomainInfo*)c->dom_d.p,
                                                                 (const uint64_t*)c->keys_sorted, (int)c->n, c->D,
                                                                 (int*)c->dranges.p);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

// Largest H per cell from the current H, deepest level first; with
// set_hlist the leaves' list radii become it plus the skins.  With particle
// lists the cell maxima are those of the particles' list extents R + s
// instead, so the cell lists hold every pair the particle lists need.
sph_status node_hmax_all(sph_ctx* c, bool set_hlist)
{
    Node* nodes = (Node*)c->nodes.p;
    const double* h = c->prm.lists == SPH_LISTS_PARTICLE && set_hlist ? (const double*)c->pext.p : c->P.H;
    for (int l = (int)c->level_off.size() - 2; l >= 0; l--) {
        const int s = c->level_off[l], nl = c->level_off[l + 1] - s;
        if (nl <= 0) continue;
        k_node_hmax<<<blocks_for(nl, 4), 256, 0, c->stream>>>(
            nodes, s, nl, h, set_hlist ? (double*)c->l_hlist.p : nullptr, c->skin_abs,
            set_hlist ? (WNode*)c->wnodes.p : nullptr);
        SPH_CHECK_LAUNCH();
    }
    return SPH_OK;
}

sph_status relist(sph_ctx* c)
{
    // particle lists: radii and skins from the current H
    if (c->prm.lists == SPH_LISTS_PARTICLE) SPH_TRY(plist_ext(c, true, nullptr));
    if (!c->radii_fresh) SPH_TRY(node_hmax_all(c, true));
    c->radii_fresh = false;
    const int nL = c->n_leaves;
    int* counts = (int*)c->l_off.p;
    int* flags = (int*)c->flags.p;
    SPH_CHECK_HIP(hipMemsetAsync(counts, 0, (size_t)(nL + 1) * sizeof(int), c->stream));
    const int with_dir = c->prm.prune == SPH_PRUNE_SORTED;
    // the gather-form force needs every leaf within either radius in both lists
    const int sym = c->prm.force_mode == SPH_FORCE_GATHER;
    // one pass into per-leaf slots, counting every entry; a slot holds about
    // twice the previous build's mean entries per leaf, and all slots together
    // at most SPH_WALK_SLOT_BYTES per particle
    int cap = c->walk_cap;
    while (cap > 16 && (size_t)nL * cap * sizeof(ListEntry) > (size_t)c->n * SPH_WALK_SLOT_BYTES) cap /= 2;
    const bool one_pass = (size_t)nL * cap * sizeof(ListEntry) <= (size_t)c->n * SPH_WALK_SLOT_BYTES + ((size_t)1 << 20);
    const int ovf_chunks = (int)std::min<int64_t>(std::max<int64_t>(1024, c->n * SPH_WALK_OVF_BYTES / (64 * 16)),
                                                  INT32_MAX / 64);
    if (one_pass) {
        SPH_TRY(buf_ensure(c->walk_scratch, (size_t)nL * cap * sizeof(ListEntry)));
        SPH_TRY(buf_ensure(c->walk_ovf, (size_t)ovf_chunks * 64 * sizeof(ListEntry)));
        SPH_TRY(buf_ensure(c->walk_link, (2 * (size_t)nL + ovf_chunks) * sizeof(int)));
        SPH_CHECK_HIP(hipMemsetAsync(flags + FI_MAXLIST, 0, sizeof(int), c->stream));
        SPH_CHECK_HIP(hipMemsetAsync(flags + FI_WOVF, 0, 2 * sizeof(int), c->stream));
        // one wave per leaf (stack entries hold node << 5)
        if (c->n_nodes < (1 << 27)) {
            k_walk_wave<<<blocks_for(nL, 4), 256, 0, c->stream>>>(
                nL, (const int*)c->leaf_node.p, (const WNode*)c->wnodes.p, (const double*)c->l_lo.p,
                (const double*)c->l_hi.p, (const int*)c->l_dom.p, (const int*)c->l_cnt.p, (const DomainInfo*)c->dom_d.p,
                (const double*)c->l_hlist.p, counts, (ListEntry*)c->walk_scratch.p, cap, with_dir, sym, flags,
                (ListEntry*)c->walk_ovf.p, (int*)c->walk_link.p, ovf_chunks);
        } else {
            k_walk<2><<<blocks_for(nL, 128), 128, 0, c->stream>>>(
                nL, (const int*)c->leaf_node.p, (const WNode*)c->wnodes.p, (const double*)c->l_lo.p,
                (const double*)c->l_hi.p, (const int*)c->l_dom.p, (const int*)c->l_cnt.p, (const DomainInfo*)c->dom_d.p,
                (const double*)c->l_hlist.p, counts, nullptr, (ListEntry*)c->walk_scratch.p, cap, with_dir, sym, flags,
                (ListEntry*)c->walk_ovf.p, (int*)c->walk_link.p, ovf_chunks);
        }
    } else {
        k_walk<0><<<blocks_for(nL, 128), 128, 0, c->stream>>>(
            nL, (const int*)c->leaf_node.p, (const WNode*)c->wnodes.p, (const double*)c->l_lo.p,
            (const double*)c->l_hi.p, (const int*)c->l_dom.p, (const int*)c->l_cnt.p, (const DomainInfo*)c->dom_d.p,
            (const double*)c->l_hlist.p, counts, nullptr, nullptr, 0, with_dir, sym, flags, nullptr, nullptr, 0);
    }
    SPH_CHECK_LAUNCH();
    SPH_TRY(scan_exclusive(c, counts, counts, nL + 1, flags + FI_NLIST));
    int hf[FI_WINC - FI_NLIST + 1];
    SPH_CHECK_HIP(hipMemcpyAsync(hf, flags + FI_NLIST, sizeof(hf), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    const int total = hf[0], incomplete = one_pass ? hf[FI_WINC - FI_NLIST] : 0;
    // particles in the fullest leaf above 64 (0: none), set by the leaf fill
    // of the last build (only a build clears the flags past FI_FLAGS)
    c->max_leaf = hf[FI_MAXLEAF - FI_NLIST];
    if (total < 0) return SPH_ERR_WORKSPACE;
    SPH_TRY(buf_ensure(c->list, (size_t)std::max(total, 1) * sizeof(ListEntry)));
    if (one_pass) {
        k_list_compact<<<blocks_for(nL, 4), 256, 0, c->stream>>>(
            nL, cap, (const ListEntry*)c->walk_scratch.p, (const ListEntry*)c->walk_ovf.p, (const int*)c->walk_link.p,
            (const int*)c->l_off.p, (ListEntry*)c->list.p);
        SPH_CHECK_LAUNCH();
    }
    if (!one_pass || incomplete > 0) {
        // leaves that found no free overflow chunk (all leaves without the
        // one pass): walked again, writing at the scanned offsets
        k_walk<1><<<blocks_for(nL, 128), 128, 0, c->stream>>>(
            nL, (const int*)c->leaf_node.p, (const WNode*)c->wnodes.p, (const double*)c->l_lo.p,
            (const double*)c->l_hi.p, (const int*)c->l_dom.p, (const int*)c->l_cnt.p, (const DomainInfo*)c->dom_d.p,
            (const double*)c->l_hlist.p, nullptr, (const int*)c->l_off.p, (ListEntry*)c->list.p, 0, with_dir, sym,
            flags, nullptr, one_pass ? (int*)c->walk_link.p : nullptr, 0);
        SPH_CHECK_LAUNCH();
    }
    // slot for the next build: the power of two at or above twice the mean
    {
        const int64_t mean2 = 2 * ((int64_t)total + nL - 1) / std::max(nL, 1);
        int nc = 16;
        while (nc < mean2 && nc < 4096) nc *= 2;
        c->walk_cap = nc;
    }
    c->n_list = total;
    c->pair_tasks_valid = false;
    // particle lists follow every new set of cell lists
    if (c->prm.lists == SPH_LISTS_PARTICLE) SPH_TRY(plist_build(c));
    return SPH_OK;
}

sph_status build_all(sph_ctx* c)
{
    const int64_t n = c->n;
    const int nd = c->prm.n_domains;
    int* flags = (int*)c->flags.p;

    // a fresh build: no displacement since the lists were made
    c->delta = 0.0;
    c->margin_h = 0.0;
    c->steps_since_build = 0;
    c->n_builds++;
    SPH_CHECK_HIP(hipMemcpyAsync(c->dparam.p, &c->margin_h, sizeof(double), hipMemcpyHostToDevice, c->stream));

    // 1. validate, per-box H range
    SPH_CHECK_HIP(hipMemsetAsync(flags, 0, FI_NFLAGS * sizeof(int), c->stream));
    std::vector<unsigned long long> dstat_h(3 * nd);
    for (int d = 0; d < nd; d++) {
        dstat_h[3 * d] = 0ull;
        dstat_h[3 * d + 2] = 0ull;
        double inf = INFINITY;
        memcpy(&dstat_h[3 * d + 1], &inf, 8);
    }
    // box extents are needed for validation before the grid is known
    c->dom_h.resize(nd);
    for (int d = 0; d < nd; d++) {
        DomainInfo& I = c->dom_h[d];
        memset(&I, 0, sizeof(I));
        for (int a = 0; a < 3; a++) I.L[a] = c->boxes[3 * d + a];
    }
    SPH_CHECK_HIP(hipMemcpyAsync(c->dom_d.p, c->dom_h.data(), nd * sizeof(DomainInfo), hipMemcpyHostToDevice, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(c->dstat.p, dstat_h.data(), 3 * nd * 8, hipMemcpyHostToDevice, c->stream));
    k_validate<<<std::min(blocks_for(n, 256), 2048), 256, 0, c->stream>>>(n, c->P.x, c->P.y, c->P.z, c->P.H, c->P.m, c->P.domain, nd,
                                                        (const DomainInfo*)c->dom_d.p,
                                                        (unsigned long long*)c->dstat.p, flags);
    SPH_CHECK_LAUNCH();
    int fl = 0;
    SPH_CHECK_HIP(hipMemcpyAsync(dstat_h.data(), c->dstat.p, 3 * nd * 8, hipMemcpyDeviceToHost, c->stream));
    SPH_TRY(read_int(c, flags, &fl));
    if (fl & FLAG_INVALID) return SPH_ERR_INVALID;
    // particle lists: the largest list radius and skin of each box
    std::vector<double> pbox;
    if (c->prm.lists == SPH_LISTS_PARTICLE) {
        pbox.assign(2 * (size_t)nd, 0.0);
        SPH_TRY(plist_ext(c, false, pbox.data()));
    }
    c->skin_max = 0.0;

    // 2. top grids (edge >= largest H of the box, >= 3 cells per dimension;
    // about twice as large where such cells would hold under 64 particles)
    int top = 0;
    double min_ratio = INFINITY;
    c->min_s0 = INFINITY;
    for (int d = 0; d < nd; d++) {
        double hmax, hmin;
        memcpy(&hmax, &dstat_h[3 * d], 8);
        memcpy(&hmin, &dstat_h[3 * d + 1], 8);
        const double nbox = (double)dstat_h[3 * d + 2];
        DomainInfo& I = c->dom_h[d];
        if (dstat_h[3 * d] == 0ull) { hmax = 0.0; hmin = INFINITY; }  // empty box
        // particle lists: top cells cover the largest list radius plus twice
        // the largest skin; where three such cells per dimension do not fit
        // the box, the allowances are scaled down by alpha until they do
        I.pl_alpha = 0.0;
        I.pl_smax = 0.0;
        if (!pbox.empty() && dstat_h[3 * d] != 0ull) {
            const double need = pbox[2 * d] + 2.0 * pbox[2 * d + 1];
            const double base = hmax * (1.0 + SPH_PLIST_SKIN);
            const double lim = std::min(I.L[0], std::min(I.L[1], I.L[2])) / 3.0;
            double alpha = 1.0;
            if (need > lim) alpha = need > base ? std::max(0.0, (lim - base) / (need - base)) : 0.0;
            alpha = std::min(alpha, 1.0);
            I.pl_alpha = alpha;
            I.pl_smax = alpha * pbox[2 * d + 1];
            hmax = std::max(hmax, std::min(lim, base + alpha * std::max(0.0, need - base)));
            c->skin_max = std::max(c->skin_max, I.pl_smax);
        }
        int ntb[3];
        for (int a = 0; a < 3; a++) {
            // largest cell count with edge L/nt >= hmax
            int nt = 3;
            if (hmax > 0.0) {
                const double q = floor(I.L[a] / hmax);
                nt = q > 1e6 ? 1000000 : (int)q;
                while (nt > 0 && I.L[a] / nt < hmax) nt--;
                while (I.L[a] / (nt + 1) >= hmax && nt < 1000000) nt++;
            }
            if (nt < 3) return SPH_ERR_BOX_TOO_SMALL;
            ntb[a] = std::min(nt, 128);
        }
        // near-uniform boxes: top cells of edge ~H hold only ~10 particles
        // each, so the leaves would stay far below a wave; there the cells
        // are taken about twice as large per dimension where the box allows
        if (nbox < 64.0 * (double)ntb[0] * ntb[1] * ntb[2])
            for (int a = 0; a < 3; a++)
                if (ntb[a] / 2 >= 3) ntb[a] /= 2;
        for (int a = 0; a < 3; a++) {
            const int nt = ntb[a];
            I.n_top[a] = nt;
            I.s0[a] = I.L[a] / nt;
            c->min_s0 = std::min(c->min_s0, I.s0[a]);
            if (hmin > 0 && std::isfinite(hmin)) min_ratio = std::min(min_ratio, hmin / I.s0[a]);
        }
        I.top_offset = top;
        top += I.n_top[0] * I.n_top[1] * I.n_top[2];
    }
    c->n_top_total = top;
    int top_bits = 1;
    while ((1ll << top_bits) < (long long)top) top_bits++;
    int D = 1;
    if (std::isfinite(min_ratio) && min_ratio > 0) D = (int)ceil(log2(1.0 / min_ratio)) + 3;
    D = std::max(1, std::min(D, SPH_MAX_DEPTH));
    D = std::min(D, (63 - top_bits) / 3);
    c->D = D;
    c->key_bits = top_bits + 3 * D;
    SPH_CHECK_HIP(hipMemcpyAsync(c->dom_d.p, c->dom_h.data(), nd * sizeof(DomainInfo), hipMemcpyHostToDevice, c->stream));

    // 3. Morton keys, radix sort, permutation of the caller's arrays
    for (int q = 0; q < 2; q++) {
        SPH_TRY(buf_ensure(c->keys[q], (size_t)n * 8));
        SPH_TRY(buf_ensure(c->vals[q], (size_t)n * 4));
    }
    k_keys<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->P.x, c->P.y, c->P.z, c->P.domain,
                                                    (const DomainInfo*)c->dom_d.p, D, (uint64_t*)c->keys[0].p,
                                                    (uint32_t*)c->vals[0].p);
    SPH_CHECK_LAUNCH();
    int res = 0;
    SPH_TRY(radix_sort(c, (int)n, c->key_bits, c->keys, c->vals, &res));
    const uint64_t* keys = (const uint64_t*)c->keys[res].p;
    c->keys_sorted = keys;
    // the other key buffer is free until the next sort: the second stream's
    // scratch; whatever path leaves this build, the stream waits for it
    struct PermJoin {
        sph_ctx* c;
        ~PermJoin() { perm_join(c); }
    } join_on_exit{c};
    SPH_TRY(permute_all(c, (const uint32_t*)c->vals[res].p, c->keys[res ^ 1].p));
    SPH_TRY(buf_ensure(c->dranges, (size_t)(nd + 1) * sizeof(int)));
    SPH_TRY(domain_ranges(c));

    // 4. octree, level by level
    size_t cap = std::max<size_t>((size_t)top * 2 + 1024, (size_t)(n / 8) + 1024);
    SPH_TRY(buf_ensure(c->nodes, cap * sizeof(Node)));
    SPH_TRY(buf_ensure(c->nchild, (size_t)(top + 1) * sizeof(int)));
    k_top_nodes<<<blocks_for(top, 256), 256, 0, c->stream>>>(top, nd, (const DomainInfo*)c->dom_d.p, keys, (int)n, D,
                                                           (Node*)c->nodes.p);
    SPH_CHECK_LAUNCH();
    // FP32 cell-relative coordinates: keep every leaf's extent within
    // SPH_FP32_EXTENT_RATIO of its smallest smoothing length
    const double h_ratio = c->prm.precision == SPH_FP64 ? 0.0 : SPH_FP32_EXTENT_RATIO;
    c->level_off.clear();
    c->level_off.push_back(0);
    int level_start = 0, n_level = top, n_nodes = top;
    c->depth = 0;
    for (int level = 0; level <= D; level++) {
        // chunks of the level: one per STATS_CHUNK particles of each cell, at
        // most n / STATS_CHUNK + the level's cells
        SPH_TRY(buf_ensure(c->lvl_cmap, ((size_t)n / STATS_CHUNK + n_level + 1) * sizeof(int)));
        SPH_TRY(buf_ensure(c->nchild, (size_t)(n_level + 1) * sizeof(int)));
        SPH_TRY(buf_ensure(c->coff, (size_t)(n_level + 1) * sizeof(int)));
        SPH_TRY(buf_ensure(c->lvl_bnd, (size_t)n_level * 9 * sizeof(int)));
        int* nchild = (int*)c->nchild.p;
        int* ccoff = (int*)c->coff.p;
        int* bnd = (int*)c->lvl_bnd.p;
        const int nbl = blocks_for(n_level, 256);
        k_level_chunks<<<nbl, 256, 0, c->stream>>>((const Node*)c->nodes.p, level_start, n_level, nchild, bnd);
        SPH_CHECK_LAUNCH();
        SPH_TRY(scan_exclusive(c, nchild, ccoff, n_level, flags + FI_NCHUNK));
        k_chunk_map<<<nbl, 256, 0, c->stream>>>(nchild, ccoff, n_level, (int*)c->lvl_cmap.p);
        SPH_CHECK_LAUNCH();
        k_level_stats<<<2048, 256, 0, c->stream>>>((Node*)c->nodes.p, level_start, level, ccoff,
                                                   (const int*)c->lvl_cmap.p, flags + FI_NCHUNK, keys, c->P.x, c->P.y,
                                                   c->P.z, c->P.H, D, bnd);
        SPH_CHECK_LAUNCH();
        k_level_split<<<nbl, 256, 0, c->stream>>>((Node*)c->nodes.p, level_start, n_level, D, c->prm.n_split, h_ratio,
                                                  bnd, nchild);
        SPH_CHECK_LAUNCH();
        SPH_TRY(scan_exclusive(c, nchild, nchild, n_level, flags + FI_NCHILD));
        // the children go at the scanned offsets, whatever their total: when
        // the node buffer holds 8 per cell of the level (the most a split
        // makes), they are written while the host reads the total
        const bool early = (size_t)n_nodes + 8 * (size_t)n_level <= cap;
        if (early) {
            k_emit_children<<<nbl, 256, 0, c->stream>>>((Node*)c->nodes.p, level_start, n_level, nchild, n_nodes, D,
                                                         c->prm.n_split, h_ratio, bnd);
            SPH_CHECK_LAUNCH();
        }
        int total = 0;
        SPH_TRY(read_int(c, flags + FI_NCHILD, &total));
        c->level_off.push_back(n_nodes);
        if (total == 0) break;
        if (!early) {
            if ((size_t)(n_nodes + total) > cap) {
                size_t ncap = std::max((size_t)(n_nodes + total) * 3 / 2, cap * 2);
                DevBuf nb2;
                SPH_TRY(buf_ensure(nb2, ncap * sizeof(Node)));
                SPH_CHECK_HIP(hipMemcpyAsync(nb2.p, c->nodes.p, (size_t)n_nodes * sizeof(Node),
                                             hipMemcpyDeviceToDevice, c->stream));
                SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
                buf_free(c->nodes);
                c->nodes = nb2;
                cap = ncap;
            }
            k_emit_children<<<nbl, 256, 0, c->stream>>>((Node*)c->nodes.p, level_start, n_level, nchild, n_nodes, D,
                                                         c->prm.n_split, h_ratio, bnd);
            SPH_CHECK_LAUNCH();
        }
        level_start = n_nodes;
        n_level = total;
        n_nodes += total;
        c->depth = level + 1;
    }
    c->n_nodes = n_nodes;

    // 5. leaves in Morton order
    SPH_TRY(buf_ensure(c->leafmark, (size_t)(n + 1) * sizeof(int)));
    SPH_CHECK_HIP(hipMemsetAsync(c->leafmark.p, 0, (size_t)(n + 1) * sizeof(int), c->stream));
    k_mark_leaves<<<blocks_for(n_nodes, 256), 256, 0, c->stream>>>((const Node*)c->nodes.p, n_nodes, (int*)c->leafmark.p);
    SPH_CHECK_LAUNCH();
    SPH_TRY(buf_ensure(c->leafscan, (size_t)(n + 1) * sizeof(int)));
    SPH_TRY(scan_exclusive(c, (const int*)c->leafmark.p, (int*)c->leafscan.p, (int)n, flags + FI_NLEAVES));
    int nL = 0;
    SPH_TRY(read_int(c, flags + FI_NLEAVES, &nL));
    c->n_leaves = nL;
    const size_t L1 = (size_t)nL + 1;
    SPH_TRY(buf_ensure(c->leaf_node, L1 * 4));
    SPH_TRY(buf_ensure(c->l_begin, L1 * 4));
    SPH_TRY(buf_ensure(c->l_count, L1 * 4));
    SPH_TRY(buf_ensure(c->l_origin, L1 * 24));
    SPH_TRY(buf_ensure(c->l_lo, L1 * 24));
    SPH_TRY(buf_ensure(c->l_hi, L1 * 24));
    SPH_TRY(buf_ensure(c->l_hlist, L1 * 8));
    SPH_TRY(buf_ensure(c->l_dom, L1 * 4));
    SPH_TRY(buf_ensure(c->l_off, (L1 + 1) * 4));
    SPH_TRY(buf_ensure(c->l_active, L1 * 4));
    SPH_TRY(buf_ensure(c->l_sorted, L1 * 4));
    SPH_TRY(buf_ensure(c->l_cnt, L1 * 4));
    k_leaf_fill<<<blocks_for(n_nodes, 256), 256, 0, c->stream>>>(
        (Node*)c->nodes.p, n_nodes, (const int*)c->leafscan.p, (int*)c->leaf_node.p, (int*)c->l_begin.p,
        (int*)c->l_count.p, (double*)c->l_origin.p, (double*)c->l_lo.p, (double*)c->l_hi.p, (double*)c->l_hlist.p,
        (int*)c->l_dom.p, (int*)c->l_cnt.p, c->skin_abs, flags + FI_MAXLEAF);
    SPH_CHECK_LAUNCH();
    // (the fullest leaf's count is read back with the list totals)

    // 6. cell-relative coordinates (the masses and every later stage need the
    // arrays permuted on the second stream)
    perm_join(c);
    const int es = c->elem_size();
    SPH_TRY(buf_ensure(c->pos4, (size_t)n * 4 * es));
    SPH_TRY(buf_ensure(c->fv4, (size_t)n * 4 * es));
    SPH_TRY(buf_ensure(c->hf, (size_t)n * es));
    if (c->prm.precision == SPH_FP64)
        k_leaf_pos<double><<<blocks_for(nL, 4), 256, 0, c->stream>>>(
            nL, (const int*)c->l_begin.p, (const int*)c->l_count.p, (const double*)c->l_origin.p, c->P.x, c->P.y,
            c->P.z, c->P.m, c->P.H, (double4*)c->pos4.p, (double*)c->hf.p);
    else
        k_leaf_pos<float><<<blocks_for(nL, 4), 256, 0, c->stream>>>(
            nL, (const int*)c->l_begin.p, (const int*)c->l_count.p, (const double*)c->l_origin.p, c->P.x, c->P.y,
            c->P.z, c->P.m, c->P.H, (float4*)c->pos4.p, (float*)c->hf.p);
    SPH_CHECK_LAUNCH();

    // 7. neighbour-cell lists (particle lists: the cell lists' radii are the
    // list extents plus the largest skin)
    if (c->prm.lists == SPH_LISTS_PARTICLE) c->skin_abs = c->skin_max;
    SPH_TRY(buf_ensure(c->wnodes, (size_t)n_nodes * sizeof(WNode)));
    k_wnodes<<<blocks_for(n_nodes, 256), 256, 0, c->stream>>>((const Node*)c->nodes.p, n_nodes, c->skin_abs,
                                                                (WNode*)c->wnodes.p);
    SPH_CHECK_LAUNCH();
    for (size_t l = 0; l + 1 < c->level_off.size(); l++) {
        const int ls = c->level_off[l], nl = c->level_off[l + 1] - ls;
        if (nl <= 0) continue;
        k_wnext<<<blocks_for(nl, 256), 256, 0, c->stream>>>((const Node*)c->nodes.p, ls, nl, (WNode*)c->wnodes.p);
        SPH_CHECK_LAUNCH();
    }
    // with cell lists the cells' largest H (octree statistics), the leaves'
    // list radii (leaf fill) and the walk nodes' bounds are those of the
    // current H: the relist need not recompute them
    c->radii_fresh = c->prm.lists == SPH_LISTS_CELL;
    SPH_TRY(relist(c));
    SPH_TRY(read_int(c, flags, &fl));
    if (fl & FLAG_INVALID) return SPH_ERR_INVALID;
    c->built = true;
    c->sorted = false;
    return SPH_OK;
}

sph_status sort_all(sph_ctx* c)
{
    // the per-direction order feeds only the sorted-axis pruning mode; with
    // box pruning the interaction kernels select candidates without it
    if (c->prm.prune != SPH_PRUNE_SORTED) {
        c->sorted = true;
        return SPH_OK;
    }
    const int64_t n = c->n;
    const int nL = c->n_leaves;
    SPH_TRY(buf_ensure(c->skey, (size_t)n * SPH_NDIR * 4));
    SPH_TRY(buf_ensure(c->sidx, (size_t)n * SPH_NDIR * 2));
    if (c->prm.precision == SPH_FP64)
        k_sort_cells<double><<<blocks_for(nL, 4), 256, 0, c->stream>>>(nL, n, (const int*)c->l_begin.p,
                                                                     (const int*)c->l_count.p, (const double4*)c->pos4.p,
                                                                     (float*)c->skey.p, (uint16_t*)c->sidx.p,
                                                                     (int*)c->l_sorted.p);
    else
        k_sort_cells<float><<<blocks_for(nL, 4), 256, 0, c->stream>>>(nL, n, (const int*)c->l_begin.p,
                                                                    (const int*)c->l_count.p, (const float4*)c->pos4.p,
                                                                    (float*)c->skey.p, (uint16_t*)c->sidx.p,
                                                                    (int*)c->l_sorted.p);
    SPH_CHECK_LAUNCH();
    c->sorted = true;
    return SPH_OK;
}

// Keep the cells and lists of the last build for a step: refresh the
// cell-relative coordinates and check every leaf against the displacement
// margin.  *fresh = false when a rebuild is needed.
// With fresh = NULL the test's flag is left on the device (the caller reads
// it together with other values) and the margin is the one on the device.
sph_status refresh_leaves(sph_ctx* c, bool* fresh)
{
    int* flags = (int*)c->flags.p;
    SPH_CHECK_HIP(hipMemsetAsync(flags, 0, sizeof(int), c->stream));
    if (fresh)
        SPH_CHECK_HIP(hipMemcpyAsync(c->dparam.p, &c->margin_h, sizeof(double), hipMemcpyHostToDevice, c->stream));
    const int nL = c->n_leaves;
    if (c->prm.precision == SPH_FP64)
        k_leaf_refresh<double><<<blocks_for(nL, 4), 256, 0, c->stream>>>(
            nL, (const int*)c->l_begin.p, (const int*)c->l_count.p, (const double*)c->l_origin.p,
            (const double*)c->l_hlist.p, (const int*)c->l_dom.p, (const DomainInfo*)c->dom_d.p, c->P.x, c->P.y, c->P.z,
            c->P.m, c->P.H, (const double*)c->dparam.p, (double4*)c->pos4.p, (double*)c->hf.p, flags,
            (const double*)c->l_lo.p, (const double*)c->l_hi.p, (const int*)c->leaf_node.p, (const Node*)c->nodes.p,
            c->D, 0.0);
    else
        k_leaf_refresh<float><<<blocks_for(nL, 4), 256, 0, c->stream>>>(
            nL, (const int*)c->l_begin.p, (const int*)c->l_count.p, (const double*)c->l_origin.p,
            (const double*)c->l_hlist.p, (const int*)c->l_dom.p, (const DomainInfo*)c->dom_d.p, c->P.x, c->P.y, c->P.z,
            c->P.m, c->P.H, (const double*)c->dparam.p, (float4*)c->pos4.p, (float*)c->hf.p, flags,
            (const double*)c->l_lo.p, (const double*)c->l_hi.p, (const int*)c->leaf_node.p, (const Node*)c->nodes.p,
            c->D, 2.0 * SPH_FP32_EXTENT_RATIO);
    SPH_CHECK_LAUNCH();
    if (!fresh) return SPH_OK;
    int fl = 0;
    SPH_TRY(read_int(c, flags, &fl));
    *fresh = !(fl & FLAG_STALE);
    return SPH_OK;
}
