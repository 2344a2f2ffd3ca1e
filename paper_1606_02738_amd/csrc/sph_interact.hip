// Density, ghost, force and integrator stages on the leaf cells.
//
// Work unit: one wave (64 lanes) per leaf cell A.  Lanes hold up to 64 of
// A's particles (i); when A holds fewer than 64 the wave is split into G
// groups of CI = 64/G lanes and group g walks every G-th neighbour of the
// staged tile, so all lanes stay busy.  A's neighbour-cell list gives the
// cells B; for each, the part of B that can be within range along the pair's
// sort direction (a window of B's sorted projections) is staged in LDS and
// streamed through.  Coordinates are cell-relative: each particle is stored
// relative to its leaf's centre, and the offset between two leaves (with the
// periodic image) is formed in FP64 once per pair of cells.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sph_ctx.h"
#include "sph_device.h"

// List entries staged per batch (NE) and the occupancy target (waves per
// SIMD, WPE) of the packed density and gather force kernels are template
// parameters chosen per context (the autotuner's tile and wave axes); the
// defaults are the measured best at 256^3 clustered.
#define SPH_DENS_WAVES 6
#define SPH_FORCEG_WAVES 5
#define SPH_BATCH 32

// Candidate buffer of the packed density path (one wave): candidates j of
// all neighbour cells in A's frame, packed 64 at a time, and A's particles.
template <typename T, int NE>
struct PTile {
    typename vec4<T>::type cand[128];  // j in A's frame, w = m
    typename vec4<T>::type si[64];     // i of A: x, y, z (A frame), H^2 (negative when inactive)
    EBatchBox<T, NE> e;
};

// Density sweep of one leaf (at most 64 particles, box pruning).  The
// candidates of every neighbour cell that pass the box test are packed into
// full tiles of 64; per tile, phase 1 runs j-major (lane = candidate, a
// uniform loop over A's active particles, one ballot per particle gives
// that particle's in-range mask) and phase 2 i-major (lane = particle,
// evaluating only the set bits).  Phase 1 keeps every lane busy whatever
// the leaf's occupancy.
template <typename T, bool COMP, int NE>
__device__ void density_leaf_packed(const DensArgs& a, int A, PTile<T, NE>& L, int lane)
{
    constexpr bool EXTRAP = sizeof(T) == 4;
    typedef typename vec4<T>::type V4;
    const V4* pos4 = (const V4*)a.pos4;
    const int bA = a.l_begin[A], nA = a.l_count[A];
    const double oA[3] = {a.l_origin[3 * A], a.l_origin[3 * A + 1], a.l_origin[3 * A + 2]};
    const DomainInfo& I = a.di[a.l_dom[A]];
    const double hlim = fmin(fmin(I.L[0], I.L[1]), I.L[2]) / 3.0;
    const double s0min = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]);
    const int e0 = a.l_off[A], e1 = a.l_off[A + 1];
    const double mg = *a.margin;  // list margin (see density_leaf)
    const double hlA = a.l_hlist[A] - mg;
    const bool vi = lane < nA;
    const int i = bA + (vi ? lane : 0);
    const bool act = vi && !a.conv[i];
    const unsigned long long amask = __ballot(act);
    if (amask == 0ull) {
        if (lane == 0) a.l_active[A] = 0;
        return;
    }
    const V4 pi = pos4[i];
    const double Hd = a.H[i];
    const T Hi = (T)Hd, H2 = Hi * Hi, invH = T(1) / Hi;
    {
        V4 q = pi;
        q.w = act ? H2 : T(-1);
        L.si[lane] = q;
    }
    Acc<T, COMP> sw, sd;
    T s2 = T(0);
    int cnt = 0;
    const double hA = wave_max(act ? Hd : 0.0);
    const T big = T(1e30);
    const T bxl = wave_min_t<T>(act ? pi.x : big), bxh = wave_max_t<T>(act ? pi.x : -big);
    const T byl = wave_min_t<T>(act ? pi.y : big), byh = wave_max_t<T>(act ? pi.y : -big);
    const T bzl = wave_min_t<T>(act ? pi.z : big), bzh = wave_max_t<T>(act ? pi.z : -big);
    const T hAm = (T)(hA * (1.0 + 1e-5));
    const T hA2 = hAm * hAm;
    auto dens_acc = [&](const V4& q4, T r2) {
        const T q = fast_sqrt(r2) * invH;
        T w, dw;
        spline_w_dw(q, w, dw);
        sw.add(q4.w * w);
        sd.add(q4.w * (T(3) * w + q * dw));
        if (EXTRAP) s2 += q4.w * spline_d2(q, dw);
        cnt++;
    };
    // box of the buffered candidates (union of their cells' boxes)
    T tlo[3] = {big, big, big}, thi[3] = {-big, -big, -big};
    // both phases on the first `len` packed candidates
    auto run_tile = [&](int len) {
        wave_sync();
        const V4 pj = L.cand[lane];
        const bool lv = lane < len;
        // particles of A farther than their H from the box of every candidate
        // have no pair in this tile
        const unsigned long long imask =
            amask & __ballot(box_d2<T>(pi.x, pi.y, pi.z, tlo[0], tlo[1], tlo[2], thi[0], thi[1], thi[2]) < H2);
        int mlo = 0, mhi = 0;
        for (unsigned long long m = imask; m; m &= m - 1ull) {
            const int ii = uniform(__ffsll((long long)m) - 1);
            const V4 q = L.si[ii];
            const T dx = pj.x - q.x, dy = pj.y - q.y, dz = pj.z - q.z;
            const unsigned long long hm = __ballot(lv && dx * dx + dy * dy + dz * dz < q.w);
            mlo = amdgcn_writelane((int)(uint32_t)hm, ii, mlo);
            mhi = amdgcn_writelane((int)(uint32_t)(hm >> 32), ii, mhi);
        }
        if (act) {
            unsigned long long m = ((unsigned long long)(uint32_t)mhi << 32) | (uint32_t)mlo;
            while (m) {
                const int s = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                const V4 q4 = L.cand[s];
                const T dx = q4.x - pi.x, dy = q4.y - pi.y, dz = q4.z - pi.z;
                dens_acc(q4, dx * dx + dy * dy + dz * dz);
            }
        }
        wave_sync();
    };
    int ncand = 0;
    // cell boxes grow by the displacement since the build plus float rounding
    const double grow = 0.5 * mg + 1e-5 * fmax(hlA, hA);
    for (int eb = e0; eb < e1; eb += NE) {
        const int nbt = min(NE, e1 - eb);
        const int nv = load_batch_box<T>(a.list, eb, nbt, lane, a.l_begin, a.l_count, a.l_origin, a.l_lo, a.l_hi,
                                         a.l_hlist, oA, I,
                                         grow, [&](const ListEntry& E) { return E.dist < hA + mg; }, L.e);
        V4 pf;  // prefetched first chunk of the next cell
        if (nv > 0 && lane < L.e.n[0]) pf = pos4[L.e.b[0] + lane];
        for (int k = 0; k < nv; k++) {
            const int bB = L.e.b[k], nB = L.e.n[k];
            const T dox = L.e.ox[k], doy = L.e.oy[k], doz = L.e.oz[k];
            const T klo[3] = {L.e.lo[0][k], L.e.lo[1][k], L.e.lo[2][k]};
            const T khi[3] = {L.e.hi[0][k], L.e.hi[1][k], L.e.hi[2][k]};
            V4 cur = pf;
            if (k + 1 < nv && lane < L.e.n[k + 1]) pf = pos4[L.e.b[k + 1] + lane];
            for (int p0 = 0; p0 < nB; p0 += 64) {
                const int len = min(64, nB - p0);
                bool in = false;
                V4 q;
                if (lane < len) {
                    q = p0 == 0 ? cur : pos4[bB + p0 + lane];
                    q.x += dox;
                    q.y += doy;
                    q.z += doz;
                    in = box_d2<T>(q.x, q.y, q.z, bxl, byl, bzl, bxh, byh, bzh) < hA2;
                }
                const unsigned long long mk = __ballot(in);
                if (in) L.cand[ncand + mask_rank(mk, lane)] = q;
                ncand += __popcll(mk);
                if (mk) {
                    for (int d = 0; d < 3; d++) {
                        tlo[d] = fmin(tlo[d], klo[d]);
                        thi[d] = fmax(thi[d], khi[d]);
                    }
                }
                if (ncand >= 64) {
                    run_tile(64);
                    const int rest = ncand - 64;
                    V4 t;
                    if (lane < rest) t = L.cand[64 + lane];
                    wave_sync();
                    if (lane < rest) L.cand[lane] = t;
                    ncand = rest;
                    // the carried candidates all come from this cell
                    for (int d = 0; d < 3; d++) {
                        tlo[d] = rest ? klo[d] : big;
                        thi[d] = rest ? khi[d] : -big;
                    }
                }
            }
        }
        wave_sync();
    }
    if (ncand > 0) run_tile(ncand);
    const bool left = dens_finish<T>(a, i, act, 0, 64, Hd, sw.total(), sd.total(), (double)s2, cnt, hlA, hlim, s0min);
    const unsigned long long lm = __ballot(left);
    if (lm && lane == 0) atomicAdd(&a.counters[CNT_UNCONV], (unsigned long long)__popcll(lm));
    if (lane == 0) a.l_active[A] = lm ? 1 : 0;
}

template <typename T, bool COMP, int PRUNE>
__device__ void density_leaf(const DensArgs& a, int A, DTile<T>& L, int lane)
{
    // FP32 modes accept a small final Newton update by second-order expansion
    constexpr bool EXTRAP = sizeof(T) == 4;
    typedef typename vec4<T>::type V4;
    const V4* pos4 = (const V4*)a.pos4;
    const int bA = a.l_begin[A], nA = a.l_count[A];
    const double oA[3] = {a.l_origin[3 * A], a.l_origin[3 * A + 1], a.l_origin[3 * A + 2]};
    const DomainInfo& I = a.di[a.l_dom[A]];
    const double hlim = fmin(fmin(I.L[0], I.L[1]), I.L[2]) / 3.0;
    const double s0min = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]);
    const int e0 = a.l_off[A], e1 = a.l_off[A + 1];
    // particles moved up to mg/2 since the lists were built: list radii shrink
    // by mg and list entries are taken up to mg farther out
    const double mg = *a.margin;
    const double hlA = a.l_hlist[A] - mg;
    bool any_left = false;
    for (int c0 = 0; c0 < nA; c0 += 64) {
        const int nc = min(64, nA - c0);
        const int lg = chunk_log2(nc);
        const int CI = 1 << lg, G = 64 >> lg;
        const int ii = lane & (CI - 1), jg = lane >> lg;
        const bool vi = ii < nc;
        const int i = bA + c0 + (vi ? ii : 0);
        const bool act = vi && !a.conv[i];
        if (__ballot(act) == 0) continue;
        const V4 pi = pos4[i];
        const double Hd = a.H[i];
        const T Hi = (T)Hd, H2 = Hi * Hi, invH = T(1) / Hi;
        Acc<T, COMP> sw, sd;
        T s2 = T(0);
        int cnt = 0;
        const double hA = wave_max(act ? Hd : 0.0);
        // bounding box of the active i (A frame) and the squared pruning radius
        const T big = T(1e30);
        const T bxl = wave_min_t<T>(act ? pi.x : big), bxh = wave_max_t<T>(act ? pi.x : -big);
        const T byl = wave_min_t<T>(act ? pi.y : big), byh = wave_max_t<T>(act ? pi.y : -big);
        const T bzl = wave_min_t<T>(act ? pi.z : big), bzh = wave_max_t<T>(act ? pi.z : -big);
        const T hAm = (T)(hA * (1.0 + 1e-5));
        const T hA2 = hAm * hAm;
        for (int eb = e0; eb < e1; eb += 64) {
            const int nbt = min(64, e1 - eb);
            const int nv = load_batch<T>(a.list, eb, nbt, lane, a.l_begin, a.l_count, a.l_origin, oA, I,
                                         [&](const ListEntry& E) { return E.dist < hA + mg; }, L.e, nullptr, A);
            V4 pf;  // prefetched first cell of the next pair
            if (PRUNE == PRUNE_BOX && nv > 0) {
                const int n0 = L.e.n[0];
                if (lane < n0) pf = pos4[L.e.b[0] + lane];
            }
            // accumulate one in-range pair (i, particle q4 of B)
            auto dens_acc = [&](const V4& q4, T r2) {
                const T q = fast_sqrt(r2) * invH;
                T w, dw;
                spline_w_dw(q, w, dw);
                sw.add(q4.w * w);
                sd.add(q4.w * (T(3) * w + q * dw));
                if (EXTRAP) s2 += q4.w * spline_d2(q, dw);
                cnt++;
            };
            // Pairs of cells in batches of NTD: phase 1 stages each neighbour
            // cell and records the in-range pairs of every lane as bits of a
            // mask; phase 2 evaluates only those pairs.
            for (int k0 = 0; k0 < nv; k0 += NTD) {
                unsigned long long msk[NTD];
                T tox[NTD], toy[NTD], toz[NTD];
#pragma unroll
                for (int u = 0; u < NTD; u++) {
                    msk[u] = 0ull;
                    tox[u] = toy[u] = toz[u] = T(0);
                    const int k = k0 + u;
                    if (k >= nv) continue;
                    const int bB = L.e.b[k], nB = L.e.n[k];
                    const T dox = L.e.ox[k], doy = L.e.oy[k], doz = L.e.oz[k];
                    tox[u] = dox;
                    toy[u] = doy;
                    toz[u] = doz;
                    const T xi = pi.x - dox, yi = pi.y - doy, zi = pi.z - doz;  // i in B's frame
                    V4* tile = L.p[u];
                    if (PRUNE == PRUNE_BOX && nB <= 64) {
                        const V4 pj = pf;
                        if (k + 1 < nv) {
                            const int n1 = L.e.n[k + 1];
                            if (lane < n1) pf = pos4[L.e.b[k + 1] + lane];
                        }
                        const bool in = lane < nB && box_d2<T>(pj.x, pj.y, pj.z, bxl - dox, byl - doy, bzl - doz,
                                                                bxh - dox, byh - doy, bzh - doz) < hA2;
                        const unsigned long long mk = __ballot(in);
                        if (in) tile[mask_rank(mk, lane)] = pj;
                        const int len = __popcll(mk);
                        wave_sync();
                        if (act) {
                            unsigned long long m = 0ull;
                            for (int s = 0, t = jg; t < len; s++, t += G) {
                                const V4 q4 = tile[t];
                                const T dx = q4.x - xi, dy = q4.y - yi, dz = q4.z - zi;
                                if (dx * dx + dy * dy + dz * dz < H2) m |= 1ull << s;
                            }
                            msk[u] = m;
                        }
                    } else {
                        // sorted-axis window (or a cell too large for one tile): one phase
                        int lo = 0, hi = nB;
                        const int dir = L.e.dir[k];
                        const bool srt = PRUNE == PRUNE_SORTED && a.l_sorted[L.e.B[k]] && nB <= 64;
                        if (srt) {
                            double uu[3];
                            sph_dir(dir, uu);
                            const float ki = (float)((double)xi * uu[0] + (double)yi * uu[1] + (double)zi * uu[2]);
                            float kmin = wave_minf(act ? ki - (float)Hd : INFINITY);
                            float kmax = wave_maxf(act ? ki + (float)Hd : -INFINITY);
                            const float eps = 1e-5f * (fabsf(kmin) + fabsf(kmax)) + 1e-6f * (float)hA;
                            sorted_window(a.skey, a.n, dir, bB, nB, lane, kmin - eps, kmax + eps, lo, hi);
                        }
                        for (int p0 = lo; p0 < hi; p0 += 64) {
                            const int len = min(64, hi - p0);
                            if (lane < len) {
                                const int t = p0 + lane;
                                const int jl = srt ? (int)a.sidx[(int64_t)dir * a.n + bB + t] : t;
                                tile[lane] = pos4[bB + jl];
                            }
                            wave_sync();
                            for (int t = jg; t < len; t += G) {
                                const V4 q4 = tile[t];
                                const T dx = q4.x - xi, dy = q4.y - yi, dz = q4.z - zi;
                                const T r2 = dx * dx + dy * dy + dz * dz;
                                if (act && r2 < H2) dens_acc(q4, r2);
                            }
                            wave_sync();
                        }
                        if (PRUNE == PRUNE_BOX && k + 1 < nv) {
                            const int n1 = L.e.n[k + 1];
                            if (lane < n1) pf = pos4[L.e.b[k + 1] + lane];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < NTD; u++) {
                    unsigned long long m = msk[u];
                    const T xi = pi.x - tox[u], yi = pi.y - toy[u], zi = pi.z - toz[u];
                    const V4* tile = L.p[u];
                    while (m) {
                        const int s = __ffsll((long long)m) - 1;
                        m &= m - 1;
                        const V4 q4 = tile[jg + G * s];
                        const T dx = q4.x - xi, dy = q4.y - yi, dz = q4.z - zi;
                        dens_acc(q4, dx * dx + dy * dy + dz * dz);
                    }
                }
                wave_sync();
            }
            wave_sync();
        }
        const bool left = dens_finish<T>(a, i, act, jg, CI, Hd, sw.total(), sd.total(), (double)s2, cnt, hlA, hlim,
                                         s0min);
        const unsigned long long lm = __ballot(left);
        if (lm) {
            any_left = true;
            if (lane == 0) atomicAdd(&a.counters[CNT_UNCONV], (unsigned long long)__popcll(lm));
        }
    }
    if (lane == 0) a.l_active[A] = any_left ? 1 : 0;
}

template <typename T, bool COMP, int PRUNE>
__global__ __launch_bounds__(256) void k_density(DensArgs a)
{
    __shared__ DTile<T> tiles[WAVES_PER_WG];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (a.gate && uniform(*a.gate) != 0) return;
    const int nL = a.nl_dev ? uniform(*a.nl_dev) : a.n_leaves;
    const int A = uniform(xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_WG + w);
    if (A >= nL) return;
    if (!a.l_active[A]) return;
    if (a.big_only && a.l_count[A] <= 64) return;
    density_leaf<T, COMP, PRUNE>(a, A, tiles[w], lane);
}


// Packed density sweep over the leaves of at most 64 particles (box
// pruning); the LDS is only the packed candidate buffer, so more waves fit
// on a CU than with the two-phase tiles.
template <typename T, bool COMP, int WPE, int NE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_density_packed(DensArgs a)
{
    __shared__ PTile<T, NE> tiles[WAVES_PER_WG];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (a.gate && uniform(*a.gate) != 0) return;
    const int nL = a.nl_dev ? uniform(*a.nl_dev) : a.n_leaves;
    const int A = uniform(xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_WG + w);
    if (A >= nL) return;
    if (!a.l_active[A] || a.l_count[A] > 64) return;
    density_leaf_packed<T, COMP, NE>(a, A, tiles[w], lane);
}

__global__ __launch_bounds__(256) void k_density_reset(int64_t n, int n_leaves, double* hlo, double* hhi, uint8_t* conv,
                                                       int* l_active, const int* nl_dev)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (nl_dev) n_leaves = *nl_dev;
    if (i < n) {
        hlo[i] = 0.0;
        hhi[i] = INFINITY;
        conv[i] = 0;
    }
    if (i < n_leaves) l_active[i] = 1;
}

// ---------------------------------------------------------------------------
// Ghost: Omega = 1 + H/(3 rho) drho/dH, P = (gamma-1) rho u, A = P/(Omega rho^2)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ghost(int64_t n, const double* __restrict__ rho, const double* __restrict__ drho,
                                               const double* __restrict__ H, const double* __restrict__ u,
                                               const double* __restrict__ vx, const double* __restrict__ vy,
                                               const double* __restrict__ vz, double gamma, double* omega, double* P,
                                               typename vec4<T>::type* fv4, T* hf, const int* gate,
                                               const double* __restrict__ ax, const double* __restrict__ ay,
                                               const double* __restrict__ az, const double* __restrict__ dudt,
                                               const double* __restrict__ hdt, int lists)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (gate && *gate != 1) return;
    // inside a step the ghost and force use v and u predicted to the end of
    // the step with the forces of its start: x + a dt/2 (hdt = dt/2; 0 outside)
    const double hd = *hdt;
    double ui = u[i], v0 = vx[i], v1 = vy[i], v2 = vz[i];
    if (hd != 0.0) {
        ui += dudt[i] * hd;
        v0 += ax[i] * hd;
        v1 += ay[i] * hd;
        v2 += az[i] * hd;
    }
    const double r = rho[i], h = H[i];
    const double om = 1.0 + h / (3.0 * r) * drho[i];
    const double p = (gamma - 1.0) * r * ui;
    const double A = p / (om * r * r);
    if (omega) omega[i] = om;
    if (P) P[i] = p;
    typename vec4<T>::type f;
    f.x = (T)v0;
    f.y = (T)v1;
    f.z = (T)v2;
    // the leaf kernels take A and H; the particle-list force takes the
    // kernel-gradient factor A (8/pi) / H^4 and 1/H directly
    f.w = lists ? (T)(A * INV_PI_8 / (h * h * h * h)) : (T)A;
    fv4[i] = f;
    hf[i] = lists ? (T)(1.0 / h) : (T)h;
}

// ---------------------------------------------------------------------------
// Force, eqs. (dvdt) and (dudt), symmetric: every unordered pair once.
// Pair cells (A,B): i-side sums in registers, j-side sums in LDS (lanes of a
// group rotate over distinct j), flushed with one atomic add per j and
// quantity.  The cell's own pairs: triangular sweep.  Each unordered pair of
// cells is evaluated by one owner: the lower index if the pair is in both
// cells' lists, else the cell whose list holds it.
// ---------------------------------------------------------------------------
struct ForceArgs {
    int n_leaves;
    int64_t n;
    const int* l_begin;
    const int* l_count;
    const double* l_origin;
    const double* l_hlist;
    const double* l_lo;
    const double* l_hi;
    const int* l_dom;
    const int* l_off;
    const ListEntry* list;
    const int* l_sorted;
    const void* pos4;
    const void* fv4;
    const void* hf;
    const float* skey;
    const uint16_t* sidx;
    const DomainInfo* di;
    double* ax;
    double* ay;
    double* az;
    double* dudt;
    int32_t* nngb;      // #{j : r_ij < H_i} incl. self at the final H (may be NULL)
    unsigned long long* counters;
    const double* margin;  // list margin: twice the largest displacement since the lists were built
    const int* gate;    // graph mode: run only if *gate == 1 (NULL: always run)
    const int* nl_dev;  // graph mode: leaf count read from the device (NULL: n_leaves)
    int persistent;
};

template <typename T> struct vec2t;
template <> struct vec2t<float> { typedef float2 type; };
template <> struct vec2t<double> { typedef double2 type; };

// One staged neighbour cell of the force stage.
template <typename T>
struct FSlots {
    typename vec4<T>::type p[64];   // x, y, z (B frame), H^2
    typename vec4<T>::type v[64];   // vx, vy, vz, k = A (8/pi) / H^4
    typename vec2t<T>::type mh[64]; // m, 1/H
    T acc[4][64];                   // j-side sums
    int jl[64];                     // local index in B
    int jn[64];                     // j-side neighbour counts (r < H_j)
};

// neighbour cells per two-phase batch (force), and the occupancy target:
// one cell per batch keeps the LDS at 6 KB per wave, and 5 waves per SIMD
// (96 VGPRs, spills outside the pair loops) measured fastest
#ifndef SPH_NTF_F32
#define SPH_NTF_F32 1
#endif
#ifndef SPH_FORCE_WAVES
#define SPH_FORCE_WAVES 5
#endif
#define NTF(T) (sizeof(T) == 4 ? SPH_NTF_F32 : 1)

template <typename T>
struct FTile {
    FSlots<T> s[NTF(T)];
    EBatch<T> e;
};

// Evaluate one pair (i, j) known to be within max(H_i, H_j); d = x_i - x_j.
// Counts the pair for i if r < H_i (and, with JSIDE, for j if r < H_j).
template <typename T, bool COMP, bool JSIDE>
__device__ inline void force_eval(T dx, T dy, T dz, T r2, T mi, T h2i, T ihi, T ki, T vxi, T vyi, T vzi,
                                  const FSlots<T>& sl, int o, FAcc<T, COMP>& ai, FSlots<T>* slw, int& ni)
{
    const typename vec4<T>::type pj = sl.p[o];
    const typename vec4<T>::type fj = sl.v[o];
    const typename vec2t<T>::type mh = sl.mh[o];
    if (r2 < h2i) ni++;
    if (JSIDE && r2 < pj.w) atomicAdd(&slw->jn[o], 1);
    if (!(r2 > T(0))) return;  // coincident particles exert no force
    const T ir = fast_rsqrt(r2);
    const T r = r2 * ir;
    const T Fi = ki * spline_dw(r * ihi);      // A_i dW/dr(r, H_i)
    const T Fj = fj.w * spline_dw(r * mh.y);   // A_j dW/dr(r, H_j)
    const T F = (Fi + Fj) * ir;
    const T dvdr = ((vxi - fj.x) * dx + (vyi - fj.y) * dy + (vzi - fj.z) * dz) * ir;
    const T mjF = mh.x * F;
    ai.ax.add(-mjF * dx);
    ai.ay.add(-mjF * dy);
    ai.az.add(-mjF * dz);
    ai.du.add(mh.x * Fi * dvdr);
    if (JSIDE) {
        const T miF = mi * F;
        atomicAdd(&slw->acc[0][o], miF * dx);
        atomicAdd(&slw->acc[1][o], miF * dy);
        atomicAdd(&slw->acc[2][o], miF * dz);
        atomicAdd(&slw->acc[3][o], mi * Fj * dvdr);
    }
}

template <typename T>
__device__ inline void stage_force_j(FSlots<T>& sl, int slot, const typename vec4<T>::type& p,
                                     const typename vec4<T>::type& f, T h, int jl)
{
    const T ih = fast_rcp(h);
    typename vec4<T>::type q = p, g = f;
    q.w = h * h;
    g.w = f.w * T(INV_PI_8) * ih * ih * ih * ih;
    typename vec2t<T>::type mh;
    mh.x = p.w;
    mh.y = ih;
    sl.p[slot] = q;
    sl.v[slot] = g;
    sl.mh[slot] = mh;
    sl.acc[0][slot] = 0;
    sl.acc[1][slot] = 0;
    sl.acc[2][slot] = 0;
    sl.acc[3][slot] = 0;
    sl.jl[slot] = jl;
    sl.jn[slot] = 0;
}

// Flush the j-side sums of a staged cell (one atomic add per particle and
// quantity; skipped for particles that received nothing).
template <typename T>
__device__ inline unsigned long long flush_j(const ForceArgs& a, const FSlots<T>& sl, int bB, int len, int lane)
{
    int jcnt = 0;
    if (lane < len) {
        const int p = bB + sl.jl[lane];
        const T gx = sl.acc[0][lane], gy = sl.acc[1][lane], gz = sl.acc[2][lane], gu = sl.acc[3][lane];
        if (gx != T(0) || gy != T(0) || gz != T(0) || gu != T(0)) {
            atomicAdd(&a.ax[p], (double)gx);
            atomicAdd(&a.ay[p], (double)gy);
            atomicAdd(&a.az[p], (double)gz);
            atomicAdd(&a.dudt[p], (double)gu);
        }
        jcnt = sl.jn[lane];
        if (jcnt && a.nngb) atomicAdd(&a.nngb[p], jcnt);
    }
    return (unsigned long long)jcnt;
}

template <typename T, bool COMP, int PRUNE>
__device__ void force_leaf(const ForceArgs& a, int A, FTile<T>& tl, int lane)
{
    typedef typename vec4<T>::type V4;
    constexpr int NT = NTF(T);
    const V4* pos4 = (const V4*)a.pos4;
    const V4* fv4 = (const V4*)a.fv4;
    const T* hf = (const T*)a.hf;
    const int bA = a.l_begin[A], nA = a.l_count[A];
    const double oA[3] = {a.l_origin[3 * A], a.l_origin[3 * A + 1], a.l_origin[3 * A + 2]};
    const DomainInfo& I = a.di[a.l_dom[A]];
    const int e0 = a.l_off[A], e1 = a.l_off[A + 1];
    const double mg = *a.margin;  // list margin (see density_leaf)
    unsigned long long npairs = 0, ndens_w = 0;
    for (int c0 = 0; c0 < nA; c0 += 64) {
        const int nc = min(64, nA - c0);
        const int lg = chunk_log2(nc);
        const int CI = 1 << lg, G = 64 >> lg;
        const int ii = lane & (CI - 1), jg = lane >> lg;
        const bool vi = ii < nc;
        const int i = bA + c0 + (vi ? ii : 0);
        const V4 pi = pos4[i];
        const V4 fi = fv4[i];
        const T Hi = hf[i];
        const T h2i = Hi * Hi, ihi = T(1) / Hi;
        const T ki = fi.w * T(INV_PI_8) * ihi * ihi * ihi * ihi;
        FAcc<T, COMP> ai;
        int nni = (jg == 0 && vi) ? 1 : 0;  // neighbour count of i, self included
        const double hA = wave_max(vi ? (double)Hi : 0.0);
        const T big = T(1e30);
        const T bxl = wave_min_t<T>(vi ? pi.x : big), bxh = wave_max_t<T>(vi ? pi.x : -big);
        const T byl = wave_min_t<T>(vi ? pi.y : big), byh = wave_max_t<T>(vi ? pi.y : -big);
        const T bzl = wave_min_t<T>(vi ? pi.z : big), bzh = wave_max_t<T>(vi ? pi.z : -big);
        FSlots<T>& s0l = tl.s[0];

        // the cell's own pairs
        if (nA <= 64) {
            // triangular sweep over the unordered pairs of the cell
            if (lane < nA) stage_force_j<T>(s0l, lane, pos4[bA + lane], fv4[bA + lane], hf[bA + lane], lane);
            wave_sync();
            const int steps = nA / 2;  // pair distances 1..floor(n/2)
            const bool even = (nA & 1) == 0;
            for (int t = jg; t < steps; t += G) {
                int b = ii + 1 + t;
                if (b >= nA) b -= nA;
                const bool ok = vi && !(even && t == steps - 1 && ii >= nA / 2);
                if (ok) {
                    const V4 pj = s0l.p[b];
                    const T dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < fmax(h2i, pj.w)) {
                        force_eval<T, COMP, true>(dx, dy, dz, r2, pi.w, h2i, ihi, ki, fi.x, fi.y, fi.z, s0l, b, ai,
                                                  &s0l, nni);
                        npairs++;
                    }
                }
            }
            wave_sync();
            if (jg == 0 && vi) {
                ai.ax.add(s0l.acc[0][ii]);
                ai.ay.add(s0l.acc[1][ii]);
                ai.az.add(s0l.acc[2][ii]);
                ai.du.add(s0l.acc[3][ii]);
                nni += s0l.jn[ii];
            }
            wave_sync();
        } else {
            // large cell: gather over all j != i of the cell (i side only)
            for (int p0 = 0; p0 < nA; p0 += 64) {
                const int len = min(64, nA - p0);
                if (lane < len) {
                    const int p = bA + p0 + lane;
                    stage_force_j<T>(s0l, lane, pos4[p], fv4[p], hf[p], p0 + lane);
                }
                wave_sync();
                for (int t = jg; t < len; t += G) {
                    if (!vi || p0 + t == c0 + ii) continue;
                    const V4 pj = s0l.p[t];
                    const T dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < fmax(h2i, pj.w)) {
                        force_eval<T, COMP, false>(dx, dy, dz, r2, pi.w, h2i, ihi, ki, fi.x, fi.y, fi.z, s0l, t,
                                                   ai, nullptr, nni);
                        if (p0 + t > c0 + ii) npairs++;
                    }
                }
                wave_sync();
            }
        }

        // pairs with other cells
        for (int eb = e0; eb < e1; eb += 64) {
            const int nbt = min(64, e1 - eb);
            const double* hl = a.l_hlist;
            const int nv = load_batch<T>(a.list, eb, nbt, lane, a.l_begin, a.l_count, a.l_origin, oA, I,
                                         [&](const ListEntry& E) {
                                             const int B = E.B;
                                             if (B == A) return false;
                                             if (B < A && E.dist < hl[B]) return false;  // owned by B
                                             return E.dist < fmax(hA + mg, hl[B]);
                                         },
                                         tl.e, hl, A);
            V4 pf, ff;
            T hh = T(1);
            if (PRUNE == PRUNE_BOX && nv > 0) {
                const int n0 = tl.e.n[0];
                if (lane < n0) {
                    const int p = tl.e.b[0] + lane;
                    pf = pos4[p];
                    ff = fv4[p];
                    hh = hf[p];
                }
            }
            for (int k0 = 0; k0 < nv; k0 += NT) {
                unsigned long long msk[NT];
                T tox[NT], toy[NT], toz[NT];
                int tlen[NT], tbB[NT];
#pragma unroll
                for (int u = 0; u < NT; u++) {
                    msk[u] = 0ull;
                    tox[u] = toy[u] = toz[u] = T(0);
                    tlen[u] = 0;
                    tbB[u] = 0;
                    const int k = k0 + u;
                    if (k >= nv) continue;
                    FSlots<T>& sl = tl.s[u];
                    const int bB = tl.e.b[k], nB = tl.e.n[k];
                    const T dox = tl.e.ox[k], doy = tl.e.oy[k], doz = tl.e.oz[k];
                    tox[u] = dox;
                    toy[u] = doy;
                    toz[u] = doz;
                    tbB[u] = bB;
                    const T xi = pi.x - dox, yi = pi.y - doy, zi = pi.z - doz;
                    if (PRUNE == PRUNE_BOX && nB <= 64) {
                        const V4 pj = pf, fj = ff;
                        const T hj = hh;
                        if (k + 1 < nv) {
                            const int n1 = tl.e.n[k + 1];
                            if (lane < n1) {
                                const int p = tl.e.b[k + 1] + lane;
                                pf = pos4[p];
                                ff = fv4[p];
                                hh = hf[p];
                            }
                        }
                        const T Rj = fmax((T)hA, hj) * T(1.00001);
                        const bool in = lane < nB && box_d2<T>(pj.x, pj.y, pj.z, bxl - dox, byl - doy, bzl - doz,
                                                                bxh - dox, byh - doy, bzh - doz) < Rj * Rj;
                        const unsigned long long mk = __ballot(in);
                        if (in) stage_force_j<T>(sl, mask_rank(mk, lane), pj, fj, hj, lane);
                        const int len = __popcll(mk);
                        tlen[u] = len;
                        wave_sync();
                        if (vi) {
                            unsigned long long m = 0ull;
                            for (int s = 0, t = jg; t < len; s++, t += G) {
                                const V4 q = sl.p[t];
                                const T dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                                if (dx * dx + dy * dy + dz * dz < fmax(h2i, q.w)) m |= 1ull << s;
                            }
                            msk[u] = m;
                            npairs += __popcll(m);
                        }
                    } else {
                        // sorted-axis window (or a cell too large for one tile): one phase
                        const T R = fmax((T)hA, tl.e.R[k]);
                        int lo = 0, hi = nB;
                        const int dir = tl.e.dir[k];
                        const bool srt = PRUNE == PRUNE_SORTED && a.l_sorted[tl.e.B[k]] && nB <= 64;
                        if (srt) {
                            double uu[3];
                            sph_dir(dir, uu);
                            const float ki_ = (float)((double)xi * uu[0] + (double)yi * uu[1] + (double)zi * uu[2]);
                            const float Rf = (float)R;
                            float kmin = wave_minf(vi ? ki_ - Rf : INFINITY);
                            float kmax = wave_maxf(vi ? ki_ + Rf : -INFINITY);
                            const float eps = 1e-5f * (fabsf(kmin) + fabsf(kmax)) + 1e-6f * Rf;
                            sorted_window(a.skey, a.n, dir, bB, nB, lane, kmin - eps, kmax + eps, lo, hi);
                        }
                        for (int p0 = lo; p0 < hi; p0 += 64) {
                            const int len = min(64, hi - p0);
                            if (lane < len) {
                                const int t = p0 + lane;
                                const int jl = srt ? (int)a.sidx[(int64_t)dir * a.n + bB + t] : t;
                                const int p = bB + jl;
                                stage_force_j<T>(sl, lane, pos4[p], fv4[p], hf[p], jl);
                            }
                            wave_sync();
                            // group jg owns slots jg, jg+G, ...; lanes of a group rotate over them
                            const int Lg = (jg < len) ? (len - jg + G - 1) / G : 0;
                            const int Lmax = (len + G - 1) / G;
                            const int s0 = (Lg > 0) ? ii % Lg : 0;
                            for (int t = 0; t < Lmax; t++) {
                                if (vi && t < Lg) {
                                    int s = s0 + t;
                                    if (s >= Lg) s -= Lg;
                                    const int o = jg + G * s;
                                    const V4 q = sl.p[o];
                                    const T dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                                    const T r2 = dx * dx + dy * dy + dz * dz;
                                    if (r2 < fmax(h2i, q.w)) {
                                        force_eval<T, COMP, true>(dx, dy, dz, r2, pi.w, h2i, ihi, ki, fi.x, fi.y,
                                                                  fi.z, sl, o, ai, &sl, nni);
                                        npairs++;
                                    }
                                }
                            }
                            wave_sync();
                            ndens_w += flush_j<T>(a, sl, bB, len, lane);
                            wave_sync();
                        }
                        if (PRUNE == PRUNE_BOX && k + 1 < nv) {
                            const int n1 = tl.e.n[k + 1];
                            if (lane < n1) {
                                const int p = tl.e.b[k + 1] + lane;
                                pf = pos4[p];
                                ff = fv4[p];
                                hh = hf[p];
                            }
                        }
                    }
                }
                // phase 2: in-range pairs only, each lane starting at its own
                // offset so that the lanes of a group touch different j
#pragma unroll
                for (int u = 0; u < NT; u++) {
                    const unsigned long long m = msk[u];
                    if (__ballot(m != 0ull) == 0ull) continue;
                    FSlots<T>& sl = tl.s[u];
                    const T xi = pi.x - tox[u], yi = pi.y - toy[u], zi = pi.z - toz[u];
                    const int len = tlen[u];
                    const int Lg = (jg < len) ? (len - jg + G - 1) / G : 0;
                    const int r0 = (Lg > 0) ? ii % Lg : 0;
                    unsigned long long mh = (r0 > 0) ? (m >> r0) : m;
                    unsigned long long ml = (r0 > 0) ? (m & ((1ull << r0) - 1ull)) : 0ull;
                    while (mh | ml) {
                        int s;
                        if (mh) {
                            s = r0 + __ffsll((long long)mh) - 1;
                            mh &= mh - 1;
                        } else {
                            s = __ffsll((long long)ml) - 1;
                            ml &= ml - 1;
                        }
                        const int o = jg + G * s;
                        const V4 q = sl.p[o];
                        const T dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                        force_eval<T, COMP, true>(dx, dy, dz, dx * dx + dy * dy + dz * dz, pi.w, h2i, ihi, ki, fi.x,
                                                  fi.y, fi.z, sl, o, ai, &sl, nni);
                    }
                }
                wave_sync();
#pragma unroll
                for (int u = 0; u < NT; u++)
                    if (tlen[u] > 0) ndens_w += flush_j<T>(a, tl.s[u], tbB[u], tlen[u], lane);
                wave_sync();
            }
            wave_sync();
        }
        double sx = ai.ax.total(), sy = ai.ay.total(), sz = ai.az.total(), su = ai.du.total();
        for (int off = CI; off < 64; off <<= 1) {
            sx += __shfl_xor(sx, off);
            sy += __shfl_xor(sy, off);
            sz += __shfl_xor(sz, off);
            su += __shfl_xor(su, off);
        }
        for (int off = CI; off < 64; off <<= 1) nni += __shfl_xor(nni, off);
        if (jg == 0 && vi) {
            atomicAdd(&a.ax[i], sx);
            atomicAdd(&a.ay[i], sy);
            atomicAdd(&a.az[i], sz);
            atomicAdd(&a.dudt[i], su);
            if (a.nngb) atomicAdd(&a.nngb[i], nni);
            ndens_w += nni;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        npairs += __shfl_xor(npairs, off);
        ndens_w += __shfl_xor(ndens_w, off);
    }
    if (lane == 0 && npairs) atomicAdd(&a.counters[CNT_NFORCE], npairs);
    if (lane == 0 && ndens_w) atomicAdd(&a.counters[CNT_NDENS_F], ndens_w);
}

template <typename T, bool COMP, int PRUNE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SPH_FORCE_WAVES, 8))) void k_force(ForceArgs a)
{
    __shared__ FTile<T> tiles[WAVES_PER_WG];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (a.gate && uniform(*a.gate) != 1) return;
    const int nL = a.nl_dev ? uniform(*a.nl_dev) : a.n_leaves;
    if (!a.persistent) {
        const int A = uniform(xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_WG + w);
        if (A >= nL) return;
        force_leaf<T, COMP, PRUNE>(a, A, tiles[w], lane);
        return;
    }
    int k = 0;
    for (int it = 0; it <= nL; it++) {
        const int A = xq_pop(&a.counters[XQ_FORCE], nL, k, lane);
        if (A < 0) break;
        force_leaf<T, COMP, PRUNE>(a, A, tiles[w], lane);
    }
}

// ---------------------------------------------------------------------------
// Gather-form force: each particle of leaf A sums its own pairs r < max(H_i,
// H_j) of eqs. (dvdt) and (dudt) over the cells of A's symmetric list.  Every
// pair is evaluated from both sides (twice the pair arithmetic of the
// pairs-once form) but nothing is accumulated on the j side, so there are no
// atomics and each output is written once.  Same packing as the density:
// candidates of all cells that pass the box test are packed 64 per tile;
// phase 1 j-major (lane = candidate, one ballot per particle of A reaching
// the tile), phase 2 i-major over the set bits.
// ---------------------------------------------------------------------------
template <typename T, int NE>
struct GTile {
    typename vec4<T>::type cp[128];   // j in A's frame: x, y, z, m
    typename vec4<T>::type cv[128];   // vx, vy, vz, k_j = A_j (8/pi) / H_j^4
    typename vec2t<T>::type ch[128];  // H_j^2, 1/H_j
    typename vec4<T>::type si[64];    // i of A: x, y, z (A frame), H_i^2 (negative: no particle)
    EBatchBox<T, NE> e;
};

template <typename T, bool COMP, int NE>
__device__ void force_leaf_gather(const ForceArgs& a, int A, GTile<T, NE>& L, int lane)
{
    typedef typename vec4<T>::type V4;
    typedef typename vec2t<T>::type V2;
    const V4* pos4 = (const V4*)a.pos4;
    const V4* fv4 = (const V4*)a.fv4;
    const T* hf = (const T*)a.hf;
    const int bA = a.l_begin[A], nA = a.l_count[A];
    const double oA[3] = {a.l_origin[3 * A], a.l_origin[3 * A + 1], a.l_origin[3 * A + 2]};
    const DomainInfo& I = a.di[a.l_dom[A]];
    const int e0 = a.l_off[A], e1 = a.l_off[A + 1];
    const double mg = *a.margin;  // list margin (see density_leaf)
    const T big = T(1e30);
    unsigned long long npairs = 0, ndens_w = 0;
    for (int c0 = 0; c0 < nA; c0 += 64) {
        const int nc = min(64, nA - c0);
        const bool vi = lane < nc;
        const int i = bA + c0 + (vi ? lane : 0);
        const unsigned long long vmask = __ballot(vi);
        const V4 pi = pos4[i];
        const V4 fi = fv4[i];
        const T Hi = hf[i];
        const T h2i = Hi * Hi, ihi = T(1) / Hi;
        const T ki = fi.w * T(INV_PI_8) * ihi * ihi * ihi * ihi;
        FAcc<T, COMP> ai;
        int nni = 0, nmax = 0;  // pairs within H_i and within max(H_i, H_j), self included
        const double hA = wave_max(vi ? (double)Hi : 0.0);
        const T hAm = (T)(hA * (1.0 + 1e-5));
        const T bxl = wave_min_t<T>(vi ? pi.x : big), bxh = wave_max_t<T>(vi ? pi.x : -big);
        const T byl = wave_min_t<T>(vi ? pi.y : big), byh = wave_max_t<T>(vi ? pi.y : -big);
        const T bzl = wave_min_t<T>(vi ? pi.z : big), bzh = wave_max_t<T>(vi ? pi.z : -big);
        wave_sync();
        {
            V4 q = pi;
            q.w = vi ? h2i : T(-1);
            L.si[lane] = q;
        }
        // box of the buffered candidates (union of their cells' boxes) and
        // the largest list radius of those cells (bounds their H)
        T tlo[3] = {big, big, big}, thi[3] = {-big, -big, -big};
        T thl = T(0);
        auto run_tile = [&](int len) {
            wave_sync();
            const V4 pj = L.cp[lane];
            const V2 hj = L.ch[lane];
            const bool lv = lane < len;
            const T R = fmax(Hi, thl) * T(1.00001);
            const unsigned long long imask =
                vmask & __ballot(box_d2<T>(pi.x, pi.y, pi.z, tlo[0], tlo[1], tlo[2], thi[0], thi[1], thi[2]) < R * R);
            int mlo = 0, mhi = 0;
            for (unsigned long long m = imask; m; m &= m - 1ull) {
                const int ii = uniform(__ffsll((long long)m) - 1);
                const V4 q = L.si[ii];
                const T dx = pj.x - q.x, dy = pj.y - q.y, dz = pj.z - q.z;
                const unsigned long long hm = __ballot(lv && dx * dx + dy * dy + dz * dz < fmax(q.w, hj.x));
                mlo = amdgcn_writelane((int)(uint32_t)hm, ii, mlo);
                mhi = amdgcn_writelane((int)(uint32_t)(hm >> 32), ii, mhi);
            }
            if (vi) {
                unsigned long long m = ((unsigned long long)(uint32_t)mhi << 32) | (uint32_t)mlo;
                while (m) {
                    const int sl = __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    const V4 q = L.cp[sl];
                    const V4 fj = L.cv[sl];
                    const V2 hh = L.ch[sl];
                    const T dx = pi.x - q.x, dy = pi.y - q.y, dz = pi.z - q.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    nmax++;
                    if (r2 < h2i) nni++;
                    // the particle itself and coincident ones exert no force:
                    // at r2 = 0 the clamp gives r = 0, dW/dr(0) = 0 and d = 0,
                    // so every term below is an exact zero (no branch)
                    const T ir = fast_rsqrt(fmax(r2, T(1e-30)));
                    const T r = r2 * ir;
                    const T Fi = ki * spline_dw(r * ihi);    // A_i dW/dr(r, H_i)
                    const T Fj = fj.w * spline_dw(r * hh.y);  // A_j dW/dr(r, H_j)
                    const T F = (Fi + Fj) * ir;
                    const T dvdr = ((fi.x - fj.x) * dx + (fi.y - fj.y) * dy + (fi.z - fj.z) * dz) * ir;
                    const T mjF = q.w * F;
                    ai.ax.add(-mjF * dx);
                    ai.ay.add(-mjF * dy);
                    ai.az.add(-mjF * dz);
                    ai.du.add(q.w * Fi * dvdr);
                }
            }
            wave_sync();
        };
        int ncand = 0;
        // cell boxes grow by the displacement since the build plus float rounding
        const double grow = 0.5 * mg + 1e-5 * hA;
        for (int eb = e0; eb < e1; eb += NE) {
            const int nbt = min(NE, e1 - eb);
            const double* hl = a.l_hlist;
            const int nv = load_batch_box<T>(a.list, eb, nbt, lane, a.l_begin, a.l_count, a.l_origin, a.l_lo, a.l_hi,
                                             hl, oA, I, grow,
                                             [&](const ListEntry& E) { return E.dist < fmax(hA + mg, hl[E.B]); }, L.e);
            // prefetched first chunk (positions, H) of the next cell
            V4 pf;
            T hp = T(1);
            if (nv > 0 && lane < L.e.n[0]) {
                const int p = L.e.b[0] + lane;
                pf = pos4[p];
                hp = hf[p];
            }
            for (int k = 0; k < nv; k++) {
                const int bB = L.e.b[k], nB = L.e.n[k];
                const T dox = L.e.ox[k], doy = L.e.oy[k], doz = L.e.oz[k];
                const V4 cq = pf;
                const T ch_ = hp;
                if (k + 1 < nv && lane < L.e.n[k + 1]) {
                    const int p = L.e.b[k + 1] + lane;
                    pf = pos4[p];
                    hp = hf[p];
                }
                for (int p0 = 0; p0 < nB; p0 += 64) {
                    const int len = min(64, nB - p0);
                    bool in = false;
                    V4 q;
                    T h = T(1);
                    if (lane < len) {
                        if (p0 == 0) {
                            q = cq;
                            h = ch_;
                        } else {
                            q = pos4[bB + p0 + lane];
                            h = hf[bB + p0 + lane];
                        }
                        q.x += dox;
                        q.y += doy;
                        q.z += doz;
                        const T Rj = fmax(hAm, h * T(1.00001));
                        in = box_d2<T>(q.x, q.y, q.z, bxl, byl, bzl, bxh, byh, bzh) < Rj * Rj;
                    }
                    const unsigned long long mk = __ballot(in);
                    if (in) {
                        const V4 f = fv4[bB + p0 + lane];
                        const int slot = ncand + mask_rank(mk, lane);
                        const T ih = fast_rcp(h);
                        V4 g = f;
                        g.w = f.w * T(INV_PI_8) * ih * ih * ih * ih;
                        V2 hh;
                        hh.x = h * h;
                        hh.y = ih;
                        L.cp[slot] = q;
                        L.cv[slot] = g;
                        L.ch[slot] = hh;
                    }
                    ncand += __popcll(mk);
                    if (mk) {
                        for (int d = 0; d < 3; d++) {
                            tlo[d] = fmin(tlo[d], L.e.lo[d][k]);
                            thi[d] = fmax(thi[d], L.e.hi[d][k]);
                        }
                        thl = fmax(thl, L.e.hl[k]);
                    }
                    if (ncand >= 64) {
                        run_tile(64);
                        const int rest = ncand - 64;
                        V4 t0, t1;
                        V2 t2;
                        if (lane < rest) {
                            t0 = L.cp[64 + lane];
                            t1 = L.cv[64 + lane];
                            t2 = L.ch[64 + lane];
                        }
                        wave_sync();
                        if (lane < rest) {
                            L.cp[lane] = t0;
                            L.cv[lane] = t1;
                            L.ch[lane] = t2;
                        }
                        ncand = rest;
                        // the carried candidates all come from this cell
                        for (int d = 0; d < 3; d++) {
                            tlo[d] = rest ? L.e.lo[d][k] : big;
                            thi[d] = rest ? L.e.hi[d][k] : -big;
                        }
                        thl = rest ? L.e.hl[k] : T(0);
                    }
                }
            }
            wave_sync();
        }
        if (ncand > 0) run_tile(ncand);
        if (vi) {
            a.ax[i] = ai.ax.total();
            a.ay[i] = ai.ay.total();
            a.az[i] = ai.az.total();
            a.dudt[i] = ai.du.total();
            if (a.nngb) a.nngb[i] = nni;
            npairs += (unsigned long long)max(nmax - 1, 0);  // ordered pairs, the particle itself excluded
            ndens_w += (unsigned long long)nni;
        }
        wave_sync();
    }
    for (int off = 32; off > 0; off >>= 1) {
        npairs += __shfl_xor(npairs, off);
        ndens_w += __shfl_xor(ndens_w, off);
    }
    if (lane == 0 && npairs) atomicAdd(&a.counters[CNT_NFORCE], npairs);
    if (lane == 0 && ndens_w) atomicAdd(&a.counters[CNT_NDENS_F], ndens_w);
}

template <typename T, bool COMP, int WPE, int NE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_force_gather(ForceArgs a)
{
    __shared__ GTile<T, NE> tiles[WAVES_PER_WG];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (a.gate && uniform(*a.gate) != 1) return;
    const int nL = a.nl_dev ? uniform(*a.nl_dev) : a.n_leaves;
    if (!a.persistent) {
        const int A = uniform(xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_WG + w);
        if (A >= nL) return;
        force_leaf_gather<T, COMP, NE>(a, A, tiles[w], lane);
        return;
    }
    int k = 0;
    for (int it = 0; it <= nL; it++) {
        const int A = xq_pop(&a.counters[XQ_FORCE], nL, k, lane);
        if (A < 0) break;
        force_leaf_gather<T, COMP, NE>(a, A, tiles[w], lane);
    }
}

// ---------------------------------------------------------------------------
// Integrator (kick-drift-kick) and FP64 conservation sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kick_drift(int64_t n, double* x, double* y, double* z, double* vx, double* vy,
                                                    double* vz, double* u, const double* __restrict__ ax,
                                                    const double* __restrict__ ay, const double* __restrict__ az,
                                                    const double* __restrict__ dudt, const int32_t* __restrict__ dom,
                                                    const DomainInfo* __restrict__ di, double dt,
                                                    unsigned long long* vmax_bits, double* H, double gm1)
{
    __shared__ double wmax[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double sp = 0.0;
    if (i < n) {
        const double h = 0.5 * dt;
        const double v[3] = {vx[i] + ax[i] * h, vy[i] + ay[i] * h, vz[i] + az[i] * h};
        vx[i] = v[0];
        vy[i] = v[1];
        vz[i] = v[2];
        const double du = dudt[i];
        const double ui = u[i] + du * h;
        u[i] = ui;
        if (H && ui > 0.0) {
            // start of the H iteration carried along the flow (see k_h_drift)
            const double e = fmin(fmax(-dt * du / (3.0 * gm1 * ui), -0.6931471805599453), 0.6931471805599453);
            H[i] *= exp(e);
        }
        sp = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const DomainInfo& I = di[dom ? dom[i] : 0];
        double* c[3] = {x, y, z};
        for (int a = 0; a < 3; a++) {
            double q = c[a][i] + v[a] * dt;
            q -= I.L[a] * floor(q / I.L[a]);
            if (q >= I.L[a]) q -= I.L[a];
            if (q < 0.0) q = 0.0;
            c[a][i] = q;
        }
    }
    // largest speed of the drift (non-negative doubles order like their bits)
    for (int off = 32; off > 0; off >>= 1) sp = fmax(sp, __shfl_xor(sp, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = sp;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmax[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) b = fmax(b, wmax[w]);
        const unsigned long long bits = (unsigned long long)__double_as_longlong(b);
        // most blocks are below the running maximum: skip their atomics
        if (bits > __atomic_load_n(vmax_bits, __ATOMIC_RELAXED)) atomicMax(vmax_bits, bits);
    }
}

// Start of the H iteration carried along the flow: with du/dt = (P/rho^2)
// drho/dt (the energy equation of Sec. 2 against the density sum) and P =
// (gamma-1) rho u, the fractional density change over dt is dt du/dt /
// ((gamma-1) u); rho H^3 stays constant, so H scales by the cube root.
__global__ __launch_bounds__(256) void k_h_drift(int64_t n, double* H, const double* __restrict__ u,
                                                 const double* __restrict__ dudt, double gm1, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ui = u[i];
    if (!(ui > 0.0)) return;
    const double e = fmin(fmax(-dt * dudt[i] / (3.0 * gm1 * ui), -0.6931471805599453), 0.6931471805599453);
    H[i] *= exp(e);
}

struct KickArgs {
    const double *ax, *ay, *az, *dudt;
    double h;  // half the step
};

// partial[(d * chunks + chunk) * 5 + k]; chunks per box is chosen so that
// the grid holds about 4096 workgroups (at least 64 per box)
// With kick != nullptr the closing half kick of the step is applied first
// (v += a dt/2, u += du/dt dt/2 with kick = {ax, ay, az, dudt}) and the
// totals are those of the kicked state.
__global__ __launch_bounds__(256) void k_sums_partial(const int* __restrict__ ranges, const double* __restrict__ m,
                                                      double* vx, double* vy, double* vz, double* u,
                                                      double* partial, int chunks, KickArgs kick)
{
    __shared__ double red[5][256];
    const int d = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
    const int b = ranges[d], e = ranges[d + 1];
    double s[5] = {0, 0, 0, 0, 0};
    for (int64_t i = b + (int64_t)ch * 256 + tid; i < e; i += (int64_t)chunks * 256) {
        if (kick.ax) {
            vx[i] += kick.ax[i] * kick.h;
            vy[i] += kick.ay[i] * kick.h;
            vz[i] += kick.az[i] * kick.h;
            u[i] += kick.dudt[i] * kick.h;
        }
        const double mm = m[i], v0 = vx[i], v1 = vy[i], v2 = vz[i];
        s[0] += mm;
        s[1] += mm * v0;
        s[2] += mm * v1;
        s[3] += mm * v2;
        s[4] += mm * (0.5 * (v0 * v0 + v1 * v1 + v2 * v2) + u[i]);
    }
    for (int k = 0; k < 5; k++) red[k][tid] = s[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st)
            for (int k = 0; k < 5; k++) red[k][tid] += red[k][tid + st];
        __syncthreads();
    }
    if (tid < 5) partial[((int64_t)d * chunks + ch) * 5 + tid] = red[tid][0];
}

// One workgroup per box: strided partial sums over the chunks, then a tree
// in LDS (fixed order, so the totals are reproducible).
__global__ __launch_bounds__(256) void k_sums_final(const double* __restrict__ partial, double* out, int chunks)
{
    __shared__ double red[5][256];
    const int d = blockIdx.x, tid = threadIdx.x;
    double s[5] = {0, 0, 0, 0, 0};
    for (int ch = tid; ch < chunks; ch += 256)
        for (int k = 0; k < 5; k++) s[k] += partial[((int64_t)d * chunks + ch) * 5 + k];
    for (int k = 0; k < 5; k++) red[k][tid] = s[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st)
            for (int k = 0; k < 5; k++) red[k][tid] += red[k][tid + st];
        __syncthreads();
    }
    if (tid < 5) out[5 * d + tid] = red[tid][0];
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
static inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

static int resident_wgs(sph_ctx* c)
{
    if (c->prm.persistent_wgs > 0) return c->prm.persistent_wgs;
    return 256 * 8;  // 256 CUs x 8 workgroups of 4 waves
}

// Leaf capacity of the per-leaf arrays: the grid of a captured launch covers
// it, and the kernels bound the work by the leaf count read on the device.
static int leaf_capacity(sph_ctx* c) { return (int)std::min<size_t>(c->l_begin.cap / sizeof(int), INT32_MAX / 2); }

static void dens_args(sph_ctx* c, const int* gate, bool graph, DensArgs& a, int& nb)
{
    memset(&a, 0, sizeof(a));
    a.n_leaves = c->n_leaves;
    a.n = c->n;
    a.l_begin = (const int*)c->l_begin.p;
    a.l_count = (const int*)c->l_count.p;
    a.l_origin = (const double*)c->l_origin.p;
    a.l_hlist = (const double*)c->l_hlist.p;
    a.l_lo = (const double*)c->l_lo.p;
    a.l_hi = (const double*)c->l_hi.p;
    a.l_dom = (const int*)c->l_dom.p;
    a.l_off = (const int*)c->l_off.p;
    a.list = (const ListEntry*)c->list.p;
    a.l_active = (int*)c->l_active.p;
    a.l_sorted = (const int*)c->l_sorted.p;
    a.pos4 = c->pos4.p;
    a.skey = (const float*)c->skey.p;
    a.sidx = (const uint16_t*)c->sidx.p;
    a.di = (const DomainInfo*)c->dom_d.p;
    a.m = c->P.m;
    a.H = c->P.H;
    a.rho = c->P.rho;
    a.drho = c->P.drho_dH;
    a.hlo = (double*)c->hlo.p;
    a.hhi = (double*)c->hhi.p;
    a.conv = (uint8_t*)c->conv.p;
    a.nngb = c->P.nngb;
    a.C_fac = pow(c->prm.kernel_gamma * c->prm.eta, 3.0);
    // FP32 sums resolve rho H^3 to about 1e-7 with compensation and a few
    // 1e-7 without; the residual test is not asked for more than that
    a.h_tol = c->prm.precision == SPH_FP64 ? c->prm.h_tol
              : std::max(c->prm.h_tol, c->prm.precision == SPH_FP32C ? SPH_FP32C_TOL_MIN : SPH_FP32_TOL_MIN);
    a.flags = (int*)c->flags.p;
    a.counters = (unsigned long long*)c->counters.p;
    a.gate = gate;
    a.margin = (const double*)c->dparam.p;
    a.nl_dev = graph ? (const int*)c->flags.p + FI_NLEAVES : nullptr;
    if (graph) a.n_leaves = 0;  // read on the device
    const int nl = graph ? leaf_capacity(c) : c->n_leaves;
    nb = blocks_for(nl, WAVES_PER_WG);
}

// The packed density and gather force kernels of the context's occupancy
// target and batch size (FP64: the defaults only).
template <typename T, bool COMP>
static void density_packed_wb(int wpe, int ne, int nb, hipStream_t s, const DensArgs& a)
{
    if (ne == 16) {
        switch (wpe) {
        case 4: k_density_packed<T, COMP, 4, 16><<<nb, 256, 0, s>>>(a); return;
        case 5: k_density_packed<T, COMP, 5, 16><<<nb, 256, 0, s>>>(a); return;
        case 8: k_density_packed<T, COMP, 8, 16><<<nb, 256, 0, s>>>(a); return;
        default: k_density_packed<T, COMP, 6, 16><<<nb, 256, 0, s>>>(a); return;
        }
    }
    switch (wpe) {
    case 4: k_density_packed<T, COMP, 4, 32><<<nb, 256, 0, s>>>(a); return;
    case 5: k_density_packed<T, COMP, 5, 32><<<nb, 256, 0, s>>>(a); return;
    case 8: k_density_packed<T, COMP, 8, 32><<<nb, 256, 0, s>>>(a); return;
    default: k_density_packed<T, COMP, 6, 32><<<nb, 256, 0, s>>>(a); return;
    }
}

static void launch_density_packed(sph_ctx* c, int nb, const DensArgs& a)
{
    const int wpe = c->prm.waves_density ? c->prm.waves_density : SPH_DENS_WAVES;
    const int ne = c->prm.batch ? c->prm.batch : SPH_BATCH;
    if (c->prm.precision == SPH_FP64) k_density_packed<double, false, SPH_DENS_WAVES, SPH_BATCH><<<nb, 256, 0, c->stream>>>(a);
    else if (c->prm.precision == SPH_FP32C) density_packed_wb<float, true>(wpe, ne, nb, c->stream, a);
    else density_packed_wb<float, false>(wpe, ne, nb, c->stream, a);
}

template <typename T, bool COMP>
static void force_gather_wb(int wpe, int ne, int nb, hipStream_t s, const ForceArgs& a)
{
    if (ne == 16) {
        switch (wpe) {
        case 4: k_force_gather<T, COMP, 4, 16><<<nb, 256, 0, s>>>(a); return;
        case 6: k_force_gather<T, COMP, 6, 16><<<nb, 256, 0, s>>>(a); return;
        case 8: k_force_gather<T, COMP, 8, 16><<<nb, 256, 0, s>>>(a); return;
        default: k_force_gather<T, COMP, 5, 16><<<nb, 256, 0, s>>>(a); return;
        }
    }
    switch (wpe) {
    case 4: k_force_gather<T, COMP, 4, 32><<<nb, 256, 0, s>>>(a); return;
    case 6: k_force_gather<T, COMP, 6, 32><<<nb, 256, 0, s>>>(a); return;
    case 8: k_force_gather<T, COMP, 8, 32><<<nb, 256, 0, s>>>(a); return;
    default: k_force_gather<T, COMP, 5, 32><<<nb, 256, 0, s>>>(a); return;
    }
}

static void launch_force_gather(sph_ctx* c, int nb, const ForceArgs& a)
{
    const int wpe = c->prm.waves_force ? c->prm.waves_force : SPH_FORCEG_WAVES;
    const int ne = c->prm.batch ? c->prm.batch : SPH_BATCH;
    if (c->prm.precision == SPH_FP64) k_force_gather<double, false, SPH_FORCEG_WAVES, SPH_BATCH><<<nb, 256, 0, c->stream>>>(a);
    else if (c->prm.precision == SPH_FP32C) force_gather_wb<float, true>(wpe, ne, nb, c->stream, a);
    else force_gather_wb<float, false>(wpe, ne, nb, c->stream, a);
}

// Density sweeps run as a grid of one wave per leaf in every execution mode:
// the persistent queues were slower here (first sweep 10.2 against 10.0 ms
// at 256^3, and the later sweeps, with most leaves converged, pay a pop per
// leaf where a grid's workgroups of converged leaves exit at once).
static sph_status launch_density(sph_ctx* c, const int* gate, bool graph = false)
{
    DensArgs a;
    int nb = 0;
    dens_args(c, gate, graph, a, nb);
    if (c->prm.lists == SPH_LISTS_PARTICLE) return launch_density_plist(c, a);
    if (nb <= 0) return SPH_OK;
    const bool srt = c->prm.prune == SPH_PRUNE_SORTED;
    if (!srt) {
        launch_density_packed(c, nb, a);
        SPH_CHECK_LAUNCH();
        // leaves above 64 particles (cells that cannot be split further):
        // the chunked two-phase kernel over a plain grid
        if (c->max_leaf <= 64) return SPH_OK;
        a.big_only = 1;
        nb = blocks_for(graph ? leaf_capacity(c) : c->n_leaves, WAVES_PER_WG);
    }
    if (c->prm.precision == SPH_FP64) {
        if (srt) k_density<double, false, PRUNE_SORTED><<<nb, 256, 0, c->stream>>>(a);
        else k_density<double, false, PRUNE_BOX><<<nb, 256, 0, c->stream>>>(a);
    } else if (c->prm.precision == SPH_FP32C) {
        if (srt) k_density<float, true, PRUNE_SORTED><<<nb, 256, 0, c->stream>>>(a);
        else k_density<float, true, PRUNE_BOX><<<nb, 256, 0, c->stream>>>(a);
    } else {
        if (srt) k_density<float, false, PRUNE_SORTED><<<nb, 256, 0, c->stream>>>(a);
        else k_density<float, false, PRUNE_BOX><<<nb, 256, 0, c->stream>>>(a);
    }
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

static sph_status density_reset(sph_ctx* c)
{
    SPH_TRY(buf_ensure(c->hlo, (size_t)c->n * 8));
    SPH_TRY(buf_ensure(c->hhi, (size_t)c->n * 8));
    SPH_TRY(buf_ensure(c->conv, (size_t)c->n));
    k_density_reset<<<blocks_for(std::max<int64_t>(c->n, c->n_leaves), 256), 256, 0, c->stream>>>(
        c->n, c->n_leaves, (double*)c->hlo.p, (double*)c->hhi.p, (uint8_t*)c->conv.p, (int*)c->l_active.p, nullptr);
    SPH_CHECK_LAUNCH();
    c->st.relists = 0;
    c->st.t_density_kernels_ms = 0.0;
    c->st.n_density_launches = 0;
    c->st.n_dens_evals = 0;
    for (int k = 0; k < 8; k++) c->st.unconv_after[k] = -1;
    return SPH_OK;
}

// Host-driven sweeps: one sweep, read the counters, relist or rebuild if a
// smoothing length outgrew the lists or the grid, repeat until converged.
// `done_sweeps` sweeps were already run on the device (graph mode).
// FP32 modes: cells are split at the build until their extent is at most
// SPH_FP32_EXTENT_RATIO times their smallest H, which bounds the error of
// the cell-relative coordinates against H.  H can shrink far below its value
// at the build during the iteration (a poor initial guess); this flags a
// leaf that could still be split and whose extent (plus the motion since
// the build) now exceeds twice that ratio times its smallest converged H.
__global__ __launch_bounds__(256) void k_extent_check(int n_leaves, const int* __restrict__ l_begin,
                                                      const int* __restrict__ l_count, const double* __restrict__ l_lo,
                                                      const double* __restrict__ l_hi, const int* __restrict__ leaf_node,
                                                      const Node* __restrict__ nodes, int max_level,
                                                      const double* __restrict__ H, double grow, int* flags)
{
    const int A = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (A >= n_leaves) return;
    const int lane = threadIdx.x & 63;
    const int b = l_begin[A], n = l_count[A];
    if (n < 2 || nodes[leaf_node[A]].level >= max_level) return;
    double hm = INFINITY;
    for (int p = b + lane; p < b + n; p += 64) hm = fmin(hm, H[p]);
    for (int off = 32; off > 0; off >>= 1) hm = fmin(hm, __shfl_xor(hm, off));
    const double ext = fmax(fmax(l_hi[3 * A] - l_lo[3 * A], l_hi[3 * A + 1] - l_lo[3 * A + 1]),
                            l_hi[3 * A + 2] - l_lo[3 * A + 2]) + grow;
    if (lane == 0 && ext > 2.0 * SPH_FP32_EXTENT_RATIO * hm) atomicOr(flags, FLAG_REBUILD);
}

static sph_status density_loop(sph_ctx* c, int done_sweeps, unsigned long long unconv0)
{
    int* flags = (int*)c->flags.p;
    unsigned long long* cnt = (unsigned long long*)c->counters.p;
    int sweeps = 0;
    unsigned long long unconv = unconv0;
    int fl = 0;
    bool prec_rebuilt = false;
    sph_status status = SPH_OK;
    for (sweeps = done_sweeps + 1; sweeps <= c->prm.max_h_iter; sweeps++) {
        SPH_CHECK_HIP(hipMemsetAsync(flags, 0, sizeof(int), c->stream));
        SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_UNCONV], 0, 8, c->stream));
        SPH_CHECK_HIP(hipEventRecord(c->kev[0], c->stream));
        SPH_TRY(launch_density(c, nullptr));
        SPH_CHECK_HIP(hipEventRecord(c->kev[1], c->stream));
        unsigned long long hc[CNT_N];
        SPH_CHECK_HIP(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
        SPH_CHECK_HIP(hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
        {
            float ms = 0.f;
            SPH_CHECK_HIP(hipEventElapsedTime(&ms, c->kev[0], c->kev[1]));
            c->st.t_density_kernels_ms += ms;
            c->st.n_density_launches++;
            c->st.n_dens_evals = (int64_t)hc[CNT_DEVAL];
        }
        unconv = hc[CNT_UNCONV];
        if (sweeps <= 8) c->st.unconv_after[sweeps - 1] = (int)std::min<unsigned long long>(unconv, INT32_MAX);
        if (fl & FLAG_BOX_SMALL) status = SPH_ERR_BOX_TOO_SMALL;
        // (inside sph_step the refresh of the next step takes this test
        // over: the lists are rebuilt then if the rule fails)
        if (unconv == 0 && c->prm.precision != SPH_FP64 && !prec_rebuilt && status == SPH_OK &&
            sweeps < c->prm.max_h_iter && !c->in_step) {
            SPH_CHECK_HIP(hipMemsetAsync(flags, 0, sizeof(int), c->stream));
            k_extent_check<<<blocks_for(c->n_leaves, 4), 256, 0, c->stream>>>(
                c->n_leaves, (const int*)c->l_begin.p, (const int*)c->l_count.p, (const double*)c->l_lo.p,
                (const double*)c->l_hi.p, (const int*)c->leaf_node.p, (const Node*)c->nodes.p, c->D, c->P.H,
                2.0 * c->delta, flags);
            SPH_CHECK_LAUNCH();
            SPH_CHECK_HIP(hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
            if (fl & FLAG_REBUILD) {
                // converged on cells too coarse for the final H: rebuild once
                // and evaluate again from the converged H
                prec_rebuilt = true;
                unconv = 1;
                SPH_TRY(build_all(c));
                SPH_TRY(sort_all(c));
                k_density_reset<<<blocks_for(std::max<int64_t>(c->n, c->n_leaves), 256), 256, 0, c->stream>>>(
                    c->n, c->n_leaves, (double*)c->hlo.p, (double*)c->hhi.p, (uint8_t*)c->conv.p,
                    (int*)c->l_active.p, nullptr);
                SPH_CHECK_LAUNCH();
                SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_NDENS], 0, 8, c->stream));
                c->st.rebuilds++;
                c->st.precision_rebuilds++;
                continue;
            }
        }
        if (unconv == 0) break;
        if ((fl & FLAG_REBUILD) || ((fl & FLAG_RELIST) && c->delta > 0.0)) {
            // a smoothing length outgrew the top grid, or outgrew its list
            // after particles moved since the build (the walk needs current
            // boxes): rebuild the cells and continue from the current H
            // (brackets restart)
            SPH_TRY(build_all(c));
            SPH_TRY(sort_all(c));
            k_density_reset<<<blocks_for(std::max<int64_t>(c->n, c->n_leaves), 256), 256, 0, c->stream>>>(
                c->n, c->n_leaves, (double*)c->hlo.p, (double*)c->hhi.p, (uint8_t*)c->conv.p, (int*)c->l_active.p, nullptr);
            SPH_CHECK_LAUNCH();
            SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_NDENS], 0, 8, c->stream));
            c->st.rebuilds++;
        } else if (fl & FLAG_RELIST) {
            SPH_TRY(relist(c));
            c->st.relists++;
        }
    }
    unsigned long long nd = 0;
    SPH_CHECK_HIP(hipMemcpyAsync(&nd, &cnt[CNT_NDENS], 8, hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    c->st.sweeps = std::min(sweeps, c->prm.max_h_iter);
    c->st.n_unconverged = (int)unconv;
    c->st.n_dens = (int64_t)nd;
    c->dens_done = true;
    c->ghost_done = false;
    c->force_done = false;
    if (status != SPH_OK) return status;
    return unconv ? SPH_ERR_NOT_CONVERGED : SPH_OK;
}

// Density stage: the first sweeps run as a gated sequence on the device (the
// same gate the graph mode uses: after each sweep a one-thread kernel turns
// the gate to "converged" or "the host must take over"), so the common case
// costs one readback for the whole stage; the host loop continues from there
// when more sweeps, a relist or a rebuild are needed.
#define SPH_GATED_SWEEPS 3

__global__ void k_graph_begin(unsigned long long* cnt, int* flags, int* gate);
__global__ void k_sweep_begin(unsigned long long* cnt, int* flags, const int* gate);
__global__ void k_sweep_end(unsigned long long* cnt, const int* flags, int* gate);

sph_status density_all(sph_ctx* c)
{
    if (!c->sorted) return SPH_ERR_STATE;
    SPH_CHECK_HIP(hipEventRecord(c->ev[0], c->stream));
    SPH_TRY(density_reset(c));
    int* gate = (int*)c->flags.p + FI_GATE;
    unsigned long long* cnt = (unsigned long long*)c->counters.p;
    int* flags = (int*)c->flags.p;
    const int sweeps = std::min(SPH_GATED_SWEEPS, c->prm.max_h_iter);
    k_graph_begin<<<1, 64, 0, c->stream>>>(cnt, flags, gate);
    SPH_CHECK_LAUNCH();
    SPH_CHECK_HIP(hipEventRecord(c->kev[0], c->stream));
    for (int k = 0; k < sweeps; k++) {
        k_sweep_begin<<<1, 64, 0, c->stream>>>(cnt, flags, gate);
        SPH_TRY(launch_density(c, gate));
        k_sweep_end<<<1, 64, 0, c->stream>>>(cnt, flags, gate);
        SPH_CHECK_LAUNCH();
    }
    SPH_CHECK_HIP(hipEventRecord(c->kev[1], c->stream));
    int hfl[FI_GATE + 1];
    unsigned long long hc[CNT_N];
    SPH_CHECK_HIP(hipMemcpyAsync(hfl, c->flags.p, sizeof(hfl), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(hc, c->counters.p, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    const int g = hfl[FI_GATE], fl = hfl[FI_FLAGS];
    const int done = (int)hc[CNT_GSWEEPS];
    {
        float ms = 0.f;
        SPH_CHECK_HIP(hipEventElapsedTime(&ms, c->kev[0], c->kev[1]));
        c->st.t_density_kernels_ms = ms;
    }
    c->st.n_density_launches = done;
    c->st.n_dens_evals = (int64_t)hc[CNT_DEVAL];
    for (int k = 0; k < 8; k++)
        c->st.unconv_after[k] = k < done && k < CNT_N - CNT_UHIST
                                    ? (int)std::min<unsigned long long>(hc[CNT_UHIST + k], INT32_MAX)
                                    : -1;
    sph_status st = SPH_OK;
    if (g == 1 && (c->prm.precision == SPH_FP64 || c->in_step)) {
        // converged (the FP32 extent check after a cold start runs in the host loop)
        c->st.sweeps = done;
        c->st.n_unconverged = 0;
        c->st.n_dens = (int64_t)hc[CNT_NDENS];
        c->dens_done = true;
        c->ghost_done = false;
        c->force_done = false;
    } else if (g == 1) {
        st = density_loop(c, done - 1, 1ull);
    } else {
        if (fl & FLAG_BOX_SMALL) {
            c->st.sweeps = done;
            c->st.n_unconverged = (int)std::min<unsigned long long>(hc[CNT_UNCONV], INT32_MAX);
            st = SPH_ERR_BOX_TOO_SMALL;
        } else {
            if ((fl & FLAG_REBUILD) || ((fl & FLAG_RELIST) && c->delta > 0.0)) {
                SPH_TRY(build_all(c));
                SPH_TRY(sort_all(c));
                k_density_reset<<<blocks_for(std::max<int64_t>(c->n, c->n_leaves), 256), 256, 0, c->stream>>>(
                    c->n, c->n_leaves, (double*)c->hlo.p, (double*)c->hhi.p, (uint8_t*)c->conv.p,
                    (int*)c->l_active.p, nullptr);
                SPH_CHECK_LAUNCH();
                SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_NDENS], 0, 8, c->stream));
                c->st.rebuilds++;
            } else if (fl & FLAG_RELIST) {
                SPH_TRY(relist(c));
                c->st.relists++;
            }
            st = density_loop(c, done, hc[CNT_UNCONV]);
        }
    }
    SPH_CHECK_HIP(hipEventRecord(c->ev[1], c->stream));
    return st;
}

static sph_status launch_ghost(sph_ctx* c, const double* u, const double* vx, const double* vy, const double* vz,
                               const int* gate)
{
    const double* hdt = (const double*)c->dparam.p + 2;
    if (c->prm.precision == SPH_FP64)
        k_ghost<double><<<blocks_for(c->n, 256), 256, 0, c->stream>>>(
            c->n, c->P.rho, c->P.drho_dH, c->P.H, u, vx, vy, vz, c->prm.gamma, c->P.omega, c->P.P, (double4*)c->fv4.p,
            (double*)c->hf.p, gate, c->P.ax, c->P.ay, c->P.az, c->P.dudt, hdt, c->prm.lists);
    else
        k_ghost<float><<<blocks_for(c->n, 256), 256, 0, c->stream>>>(
            c->n, c->P.rho, c->P.drho_dH, c->P.H, u, vx, vy, vz, c->prm.gamma, c->P.omega, c->P.P, (float4*)c->fv4.p,
            (float*)c->hf.p, gate, c->P.ax, c->P.ay, c->P.az, c->P.dudt, hdt, c->prm.lists);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

// Half step of the velocity and energy prediction the ghost applies (a step
// in progress) or 0, uploaded to the device slot the ghost reads.
static sph_status set_prediction(sph_ctx* c)
{
    c->hdt_up = c->predicted ? c->hdt_h : 0.0;
    SPH_CHECK_HIP(hipMemcpyAsync((double*)c->dparam.p + 2, &c->hdt_up, sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
    return SPH_OK;
}

sph_status ghost_all(sph_ctx* c)
{
    if (!c->dens_done) return SPH_ERR_STATE;
    const double *u = c->P.u, *vx = c->P.vx, *vy = c->P.vy, *vz = c->P.vz;
    SPH_TRY(set_prediction(c));
    SPH_CHECK_HIP(hipEventRecord(c->ev[2], c->stream));
    SPH_TRY(launch_ghost(c, u, vx, vy, vz, nullptr));
    SPH_CHECK_HIP(hipEventRecord(c->ev[3], c->stream));
    c->ghost_done = true;
    return SPH_OK;
}

static void force_args(sph_ctx* c, const int* gate, bool graph, ForceArgs& a, int& nb)
{
    memset(&a, 0, sizeof(a));
    a.n_leaves = c->n_leaves;
    a.n = c->n;
    a.l_begin = (const int*)c->l_begin.p;
    a.l_count = (const int*)c->l_count.p;
    a.l_origin = (const double*)c->l_origin.p;
    a.l_hlist = (const double*)c->l_hlist.p;
    a.l_lo = (const double*)c->l_lo.p;
    a.l_hi = (const double*)c->l_hi.p;
    a.l_dom = (const int*)c->l_dom.p;
    a.l_off = (const int*)c->l_off.p;
    a.list = (const ListEntry*)c->list.p;
    a.l_sorted = (const int*)c->l_sorted.p;
    a.pos4 = c->pos4.p;
    a.fv4 = c->fv4.p;
    a.hf = c->hf.p;
    a.skey = (const float*)c->skey.p;
    a.sidx = (const uint16_t*)c->sidx.p;
    a.di = (const DomainInfo*)c->dom_d.p;
    a.ax = c->P.ax;
    a.ay = c->P.ay;
    a.az = c->P.az;
    a.dudt = c->P.dudt;
    a.nngb = c->P.nngb;
    a.counters = (unsigned long long*)c->counters.p;
    a.persistent = c->prm.exec_mode == SPH_EXEC_PERSISTENT;
    a.gate = gate;
    a.margin = (const double*)c->dparam.p;
    a.nl_dev = graph ? (const int*)c->flags.p + FI_NLEAVES : nullptr;
    if (graph) a.n_leaves = 0;  // read on the device
    const int nl = graph ? leaf_capacity(c) : c->n_leaves;
    nb = a.persistent ? std::min(resident_wgs(c), blocks_for(nl, WAVES_PER_WG)) : blocks_for(nl, WAVES_PER_WG);
}

static sph_status launch_force(sph_ctx* c, const int* gate, bool graph = false)
{
    if (c->prm.lists == SPH_LISTS_PARTICLE) return launch_force_plist(c, gate);
    ForceArgs a;
    int nb = 0;
    force_args(c, gate, graph, a, nb);
    if (nb > 0 && c->prm.force_mode == SPH_FORCE_GATHER) {
        launch_force_gather(c, nb, a);
        SPH_CHECK_LAUNCH();
    } else if (nb > 0) {
        const bool srt = c->prm.prune == SPH_PRUNE_SORTED;
        if (c->prm.precision == SPH_FP64) {
            if (srt) k_force<double, false, PRUNE_SORTED><<<nb, 256, 0, c->stream>>>(a);
            else k_force<double, false, PRUNE_BOX><<<nb, 256, 0, c->stream>>>(a);
        } else if (c->prm.precision == SPH_FP32C) {
            if (srt) k_force<float, true, PRUNE_SORTED><<<nb, 256, 0, c->stream>>>(a);
            else k_force<float, true, PRUNE_BOX><<<nb, 256, 0, c->stream>>>(a);
        } else {
            if (srt) k_force<float, false, PRUNE_SORTED><<<nb, 256, 0, c->stream>>>(a);
            else k_force<float, false, PRUNE_BOX><<<nb, 256, 0, c->stream>>>(a);
        }
        SPH_CHECK_LAUNCH();
    }
    return SPH_OK;
}

// Running totals of the interaction counters (device, no host round trip):
// the force stage's N_force (ordered, as counted) and N_dens are added to
// CNT_NFORCE_SUM / CNT_NDENS_SUM after every force launch.
__global__ void k_count_totals(unsigned long long* cnt, const int* gate)
{
    if (gate && *gate != 1) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt[CNT_NFORCE_SUM] += cnt[CNT_NFORCE];
        cnt[CNT_NDENS_SUM] += cnt[CNT_NDENS_F];
        cnt[CNT_FORCE_CALLS] += 1ull;
    }
}

// Force stage, asynchronous: the counts and the kernel's duration are read by
// sph_get_stats (force_pending).
sph_status force_all(sph_ctx* c)
{
    if (!c->ghost_done) return SPH_ERR_STATE;
    const size_t nb8 = (size_t)c->n * 8;
    unsigned long long* cnt = (unsigned long long*)c->counters.p;
    SPH_CHECK_HIP(hipEventRecord(c->ev[4], c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(c->P.ax, 0, nb8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(c->P.ay, 0, nb8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(c->P.az, 0, nb8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(c->P.dudt, 0, nb8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_NFORCE], 0, 8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(&cnt[XQ_FORCE], 0, XQ_N * XQ_STRIDE * 8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_NDENS_F], 0, 8, c->stream));
    if (c->P.nngb) SPH_CHECK_HIP(hipMemsetAsync(c->P.nngb, 0, (size_t)c->n * 4, c->stream));
    SPH_CHECK_HIP(hipEventRecord(c->kev[2], c->stream));
    SPH_TRY(launch_force(c, nullptr));
    SPH_CHECK_HIP(hipEventRecord(c->kev[3], c->stream));
    k_count_totals<<<1, 64, 0, c->stream>>>(cnt, nullptr);
    SPH_CHECK_LAUNCH();
    SPH_CHECK_HIP(hipEventRecord(c->ev[5], c->stream));
    c->force_pending = true;
    c->force_done = true;
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Graph mode: density sweeps, ghost and force captured in one hipGraph.  The
// sweep count is data dependent, so the graph holds a fixed number of sweeps
// gated by a device flag: 0 = sweeping, 1 = converged (the remaining sweeps
// exit at once, ghost and force run), 2 = the host must take over (lists or
// grid need rebuilding, or H hit the box limit; ghost and force are skipped).
// Counters and outputs are cleared by kernels, not memset nodes.  Grids cover
// the leaf capacity and the kernels read the leaf count from the device, so
// one graph serves every rebuild that keeps the buffers in place; it is
// captured again when any kernel argument changes.
// ---------------------------------------------------------------------------
#define SPH_GRAPH_SWEEPS 4

__global__ void k_graph_begin(unsigned long long* cnt, int* flags, int* gate)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        // the force stage's counters are left to the force stage (they may
        // still be unread by the host)
        cnt[CNT_UNCONV] = 0ull;
        cnt[CNT_NDENS] = 0ull;
        cnt[CNT_DEVAL] = 0ull;
        cnt[CNT_GSWEEPS] = 0ull;
        for (int k = CNT_UHIST; k < CNT_N; k++) cnt[k] = 0ull;
        flags[FI_FLAGS] = 0;
        *gate = 0;
    }
}

__global__ void k_sweep_begin(unsigned long long* cnt, int* flags, const int* gate)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && *gate == 0) {
        cnt[CNT_UNCONV] = 0ull;
        flags[FI_FLAGS] = 0;
        cnt[CNT_GSWEEPS] += 1ull;
    }
}

// same decision order as the host loop: box limit, converged, rebuild/relist
__global__ void k_sweep_end(unsigned long long* cnt, const int* flags, int* gate)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && *gate == 0) {
        const int f = flags[FI_FLAGS];
        const unsigned long long k = cnt[CNT_GSWEEPS];
        if (k >= 1 && k <= CNT_N - CNT_UHIST) cnt[CNT_UHIST + k - 1] = cnt[CNT_UNCONV];
        if (f & FLAG_BOX_SMALL) *gate = 2;
        else if (cnt[CNT_UNCONV] == 0ull) *gate = 1;
        else if (f & (FLAG_RELIST | FLAG_REBUILD)) *gate = 2;
    }
}

__global__ __launch_bounds__(256) void k_force_zero(int64_t n, double* ax, double* ay, double* az, double* dudt,
                                                    int32_t* nngb, unsigned long long* cnt, const int* gate)
{
    if (*gate != 1) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        cnt[CNT_NFORCE] = 0ull;
        for (int r = 0; r < XQ_N; r++) cnt[XQ_FORCE + r * XQ_STRIDE] = 0ull;
        cnt[CNT_NDENS_F] = 0ull;
    }
    if (i < n) {
        ax[i] = 0.0;
        ay[i] = 0.0;
        az[i] = 0.0;
        dudt[i] = 0.0;
        if (nngb) nngb[i] = 0;
    }
}

template <typename X>
static void key_put(std::vector<uint8_t>& k, const X& x)
{
    const uint8_t* p = (const uint8_t*)&x;
    k.insert(k.end(), p, p + sizeof(X));
}

// Every argument and grid size the graph's launches would take now.
static std::vector<uint8_t> graph_key(sph_ctx* c, const double* u, const double* vx, const double* vy,
                                      const double* vz, int sweeps)
{
    const int* gate = (const int*)c->flags.p + FI_GATE;
    std::vector<uint8_t> k;
    DensArgs da;
    ForceArgs fa;
    int nbd = 0, nbf = 0;
    dens_args(c, gate, true, da, nbd);
    force_args(c, gate, true, fa, nbf);
    key_put(k, da);
    key_put(k, fa);
    key_put(k, nbd);
    key_put(k, nbf);
    key_put(k, sweeps);
    key_put(k, c->n);
    key_put(k, leaf_capacity(c));
    const void* ptrs[] = {u, vx, vy, vz, c->hlo.p, c->hhi.p, c->conv.p, c->l_active.p, c->P.omega, c->P.P, c->fv4.p,
                          c->hf.p, c->P.rho, c->P.drho_dH, c->P.H, c->stream};
    key_put(k, ptrs);
    key_put(k, c->prm.precision);
    key_put(k, c->prm.prune);
    key_put(k, c->prm.exec_mode);
    key_put(k, (int)(c->max_leaf > 64));  // whether the big-leaf density pass is launched
    const void* pptrs[] = {c->pq.p, c->pR.p, c->plen.p, c->plist.p, c->prem.p, c->ch_p0.p, c->ch_n.p,
                           c->ch_uo.p, c->ch_ro.p, c->ch_U.p, c->P.domain, c->P.nngb};
    key_put(k, pptrs);
    key_put(k, c->n_chunks);
    key_put(k, c->prm.lists);
    key_put(k, c->prm.tile);
    key_put(k, c->prm.waves_density);
    key_put(k, c->prm.waves_force);
    key_put(k, c->prm.batch);
    return k;
}

static sph_status capture_dgf(sph_ctx* c, const double* u, const double* vx, const double* vy, const double* vz,
                              int sweeps)
{
    if (c->graph_exec) {
        (void)hipGraphExecDestroy((hipGraphExec_t)c->graph_exec);
        c->graph_exec = nullptr;
    }
    c->graph_key.clear();
    // the caller's stream may be the legacy default stream, which cannot be
    // captured: record on a private stream, launch on the caller's
    if (!c->cap_stream) SPH_CHECK_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    int* gate = (int*)c->flags.p + FI_GATE;
    unsigned long long* cnt = (unsigned long long*)c->counters.p;
    int* flags = (int*)c->flags.p;
    const int* nl_dev = (const int*)c->flags.p + FI_NLEAVES;
    const int nlc = leaf_capacity(c);
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        c->stream = user;
        return SPH_ERR_HIP;
    }
    sph_status st = SPH_OK;
    k_density_reset<<<blocks_for(std::max<int64_t>(c->n, nlc), 256), 256, 0, c->stream>>>(
        c->n, nlc, (double*)c->hlo.p, (double*)c->hhi.p, (uint8_t*)c->conv.p, (int*)c->l_active.p, nl_dev);
    k_graph_begin<<<1, 64, 0, c->stream>>>(cnt, flags, gate);
    for (int k = 0; k < sweeps && st == SPH_OK; k++) {
        k_sweep_begin<<<1, 64, 0, c->stream>>>(cnt, flags, gate);
        st = launch_density(c, gate, true);
        k_sweep_end<<<1, 64, 0, c->stream>>>(cnt, flags, gate);
    }
    if (st == SPH_OK) st = launch_ghost(c, u, vx, vy, vz, gate);
    k_force_zero<<<blocks_for(c->n, 256), 256, 0, c->stream>>>(c->n, c->P.ax, c->P.ay, c->P.az, c->P.dudt, c->P.nngb,
                                                              cnt, gate);
    if (st == SPH_OK) st = launch_force(c, gate, true);
    k_count_totals<<<1, 64, 0, c->stream>>>(cnt, gate);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->stream = user;
    if (st != SPH_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st != SPH_OK ? st : SPH_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return SPH_ERR_HIP;
    c->graph_exec = ex;
    c->graph_key = graph_key(c, u, vx, vy, vz, sweeps);
    c->st.graph_captures++;
    return SPH_OK;
}

// Density, ghost and force through the captured graph; the host finishes
// whatever the graph could not (more sweeps, list or grid rebuilds).
sph_status dgf_graph(sph_ctx* c)
{
    if (!c->sorted) return SPH_ERR_STATE;
    const double *u = c->P.u, *vx = c->P.vx, *vy = c->P.vy, *vz = c->P.vz;
    SPH_TRY(set_prediction(c));
    SPH_TRY(buf_ensure(c->hlo, (size_t)c->n * 8));
    SPH_TRY(buf_ensure(c->hhi, (size_t)c->n * 8));
    SPH_TRY(buf_ensure(c->conv, (size_t)c->n));
    const int sweeps = std::min(SPH_GRAPH_SWEEPS, c->prm.max_h_iter);
    if (!c->graph_exec || c->graph_key != graph_key(c, u, vx, vy, vz, sweeps))
        SPH_TRY(capture_dgf(c, u, vx, vy, vz, sweeps));
    c->st.relists = 0;
    c->st.n_density_launches = 0;
    c->st.n_dens_evals = 0;
    for (int k = 0; k < 8; k++) c->st.unconv_after[k] = -1;
    SPH_CHECK_HIP(hipEventRecord(c->ev[0], c->stream));
    SPH_CHECK_HIP(hipGraphLaunch((hipGraphExec_t)c->graph_exec, c->stream));
    SPH_CHECK_HIP(hipEventRecord(c->ev[1], c->stream));
    int hfl[FI_GATE + 1];
    unsigned long long hc[CNT_N];
    SPH_CHECK_HIP(hipMemcpyAsync(hfl, c->flags.p, sizeof(hfl), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(hc, c->counters.p, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    const int gate = hfl[FI_GATE], fl = hfl[FI_FLAGS];
    const int gsweeps = (int)hc[CNT_GSWEEPS];
    // the graph's kernels are not timed one by one
    c->st.t_density_kernels_ms = -1.0;
    c->st.t_force_kernel_ms = -1.0;
    c->st.n_density_launches = gsweeps;
    c->st.n_dens_evals = (int64_t)hc[CNT_DEVAL];
    for (int k = 0; k < 8; k++)
        c->st.unconv_after[k] = k < gsweeps && k < CNT_N - CNT_UHIST
                                    ? (int)std::min<unsigned long long>(hc[CNT_UHIST + k], INT32_MAX)
                                    : -1;
    if (gate == 1) {
        c->st.sweeps = gsweeps;
        c->st.n_unconverged = 0;
        c->st.n_force = (int64_t)(c->prm.force_mode == SPH_FORCE_GATHER ? hc[CNT_NFORCE] / 2 : hc[CNT_NFORCE]);
        c->st.n_dens = (int64_t)hc[CNT_NDENS_F];
        c->dens_done = c->ghost_done = c->force_done = true;
        // the whole graph is accounted as the density stage
        for (int k = 2; k < 6; k++) SPH_CHECK_HIP(hipEventRecord(c->ev[k], c->stream));
        return SPH_OK;
    }
    // the host takes over from the state the graph left
    c->st.graph_fallbacks++;
    if (fl & FLAG_BOX_SMALL) return SPH_ERR_BOX_TOO_SMALL;
    if ((fl & FLAG_REBUILD) || ((fl & FLAG_RELIST) && c->delta > 0.0)) {
        SPH_TRY(build_all(c));
        SPH_TRY(sort_all(c));
        k_density_reset<<<blocks_for(std::max<int64_t>(c->n, c->n_leaves), 256), 256, 0, c->stream>>>(
            c->n, c->n_leaves, (double*)c->hlo.p, (double*)c->hhi.p, (uint8_t*)c->conv.p, (int*)c->l_active.p,
            nullptr);
        SPH_CHECK_LAUNCH();
        SPH_CHECK_HIP(hipMemsetAsync(&((unsigned long long*)c->counters.p)[CNT_NDENS], 0, 8, c->stream));
        c->st.rebuilds++;
    } else if (fl & FLAG_RELIST) {
        SPH_TRY(relist(c));
        c->st.relists++;
    }
    sph_status s = density_loop(c, gsweeps, hc[CNT_UNCONV]);
    c->st.t_density_kernels_ms = -1.0;
    SPH_CHECK_HIP(hipEventRecord(c->ev[1], c->stream));
    if (s != SPH_OK) return s;
    SPH_TRY(ghost_all(c));
    return force_all(c);
}

static sph_status sums_impl(sph_ctx* c, double* host_out, KickArgs kick)
{
    const int nd = c->prm.n_domains;
    // one 256-thread workgroup per chunk of a box; at most one chunk per 1024
    // particles (>= 4 per thread) and about 4096 chunks over all boxes
    const int chunks = (int)std::max<int64_t>(
        1, std::min<int64_t>(std::max(64, 4096 / std::max(nd, 1)), (c->n + 1023) / 1024));
    SPH_TRY(buf_ensure(c->dsum_part, (size_t)nd * chunks * 5 * 8 + (size_t)nd * 5 * 8));
    const int* ranges = (const int*)c->dranges.p;
    double* part = (double*)c->dsum_part.p;
    double* out = part + (size_t)nd * chunks * 5;
    dim3 g(chunks, nd);
    k_sums_partial<<<g, 256, 0, c->stream>>>(ranges, c->P.m, c->P.vx, c->P.vy, c->P.vz, c->P.u, part, chunks, kick);
    SPH_CHECK_LAUNCH();
    k_sums_final<<<nd, 256, 0, c->stream>>>(part, out, chunks);
    SPH_CHECK_LAUNCH();
    c->sums_dev = out;
    if (!host_out) {
        c->sums_pending = true;  // read by sph_get_stats
        return SPH_OK;
    }
    SPH_CHECK_HIP(hipMemcpyAsync(host_out, out, (size_t)nd * 5 * 8, hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    return SPH_OK;
}

sph_status domain_sums(sph_ctx* c, double* host_out)
{
    KickArgs none{};
    return sums_impl(c, host_out, none);
}

static sph_status step_impl(sph_ctx* c, double dt);

// Particle lists built inside the step (cell rebuilds and relists) size their
// skins and growth allowances for rebuild_steps steps of this length.
sph_status step_all(sph_ctx* c, double dt)
{
    c->list_dt = dt;
    const sph_status s = step_impl(c, dt);
    c->list_dt = 0.0;
    return s;
}

// Displacement bound of the kept lists, on the device: margin += 2 vmax dt.
__global__ void k_margin(double* dparam, double dt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double v;
        const unsigned long long b = ((const unsigned long long*)dparam)[1];
        memcpy(&v, &b, 8);
        dparam[0] += 2.0 * v * dt;
    }
}

// One step.  The host reads the device once before the density stage (the
// step's largest speed and whether the kept cells and lists are still valid:
// the cell build is host-driven) and once inside the density stage; the
// force, the closing kick and the FP64 totals are enqueued without waiting
// (the totals are read by sph_get_stats).
static sph_status step_impl(sph_ctx* c, double dt)
{
    if (!c->force_done) return SPH_ERR_STATE;
    const int nb = blocks_for(c->n, 256);
    unsigned long long* vmax_bits = (unsigned long long*)c->dparam.p + 1;
    SPH_CHECK_HIP(hipMemsetAsync(vmax_bits, 0, 8, c->stream));
    // the start of the H iteration is carried along the flow unless the
    // predictor supplies it; fused into the kick-drift unless the predictor
    // records samples (its features read the H before the drift)
    const bool drift = c->prm.h_drift && !(c->h_pred && c->mlp_ready);
    const bool fuse = drift && !c->rec_on;
    k_kick_drift<<<nb, 256, 0, c->stream>>>(c->n, c->P.x, c->P.y, c->P.z, c->P.vx, c->P.vy, c->P.vz, c->P.u, c->P.ax,
                                            c->P.ay, c->P.az, c->P.dudt, c->P.domain, (const DomainInfo*)c->dom_d.p,
                                            dt, vmax_bits, fuse ? c->P.H : nullptr, c->prm.gamma - 1.0);
    SPH_CHECK_LAUNCH();
    c->step_count++;
    SPH_TRY(mlp_pre_build(c, dt));
    if (drift && !fuse) {
        k_h_drift<<<nb, 256, 0, c->stream>>>(c->n, c->P.H, c->P.u, c->P.dudt, c->prm.gamma - 1.0, dt);
        SPH_CHECK_LAUNCH();
    }
    SPH_CHECK_HIP(hipEventRecord(c->ev[6], c->stream));
    const bool keep = c->prm.rebuild_steps > 0 && c->built;
    if (keep) {
        // keep the cells and lists while the displacement margin allows
        k_margin<<<1, 64, 0, c->stream>>>((double*)c->dparam.p, dt);
        SPH_CHECK_LAUNCH();
        if (c->prm.lists == SPH_LISTS_PARTICLE) SPH_TRY(plist_refresh(c, nullptr));
        else SPH_TRY(refresh_leaves(c, nullptr));
    }
    double dp[2] = {0.0, 0.0};
    int fl = 0;
    SPH_CHECK_HIP(hipMemcpyAsync(dp, c->dparam.p, 16, hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(&fl, c->flags.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if (keep && c->prm.lists == SPH_LISTS_PARTICLE)
        SPH_CHECK_HIP(hipMemcpyAsync(c->stale_h, (unsigned long long*)c->counters.p + CNT_STALE_MOVED, 16,
                                     hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    double vmax;
    {
        unsigned long long b;
        memcpy(&b, &dp[1], 8);
        memcpy(&vmax, &b, 8);
    }
    bool fresh = false;
    if (keep) {
        c->margin_h = dp[0];
        c->delta = 0.5 * dp[0];
        fresh = !(fl & FLAG_STALE);
        if (c->prm.lists == SPH_LISTS_PARTICLE) {
            c->st.stale_moved = (int64_t)c->stale_h[0];
            c->st.stale_grown = (int64_t)c->stale_h[1];
        }
    }
    if (fresh) {
        c->steps_since_build++;
    } else {
        // list skin for the coming steps: rebuild_steps times this step's
        // largest displacement
        c->skin_abs = c->prm.rebuild_steps > 0 ? c->prm.rebuild_steps * vmax * dt : 0.0;
        // the density and ghost stages below write rho, drho_dH, omega and P
        // of every particle (all start unconverged) before anything reads them
        c->dens_outputs_dead = true;
        const sph_status sb = build_all(c);
        c->dens_outputs_dead = false;
        SPH_TRY(sb);
    }
    SPH_TRY(sort_all(c));
    SPH_CHECK_HIP(hipEventRecord(c->ev[7], c->stream));
    sph_status s;
    c->hdt_h = 0.5 * dt;
    c->predicted = true;
    c->in_step = true;
    if (c->prm.use_graph) {
        s = dgf_graph(c);
    } else {
        s = density_all(c);
        if (s == SPH_OK) s = ghost_all(c);
        if (s == SPH_OK) s = force_all(c);
    }
    c->predicted = false;
    c->in_step = false;
    if (s != SPH_OK) return s;
    SPH_TRY(mlp_post_step(c));
    // closing half kick, fused with the FP64 totals of the kicked state
    KickArgs kick{c->P.ax, c->P.ay, c->P.az, c->P.dudt, 0.5 * dt};
    SPH_TRY(sums_impl(c, nullptr, kick));
    return SPH_OK;
}
