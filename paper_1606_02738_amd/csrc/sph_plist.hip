// Per-particle neighbour lists (lists = SPH_LISTS_PARTICLE).
//
// The cells and their neighbour-cell lists (Sec. 3.1) decide which particles
// can interact; this file turns them, once per cell build, into one list per
// particle of the candidates j with r_ij < max(R_i, R_j) + s_i + s_j, where
// R = 1.02 H is the particle's list radius and s its skin: the distance it
// may move before the lists are rebuilt, from its own speed and acceleration
// over rebuild_steps steps.  The lists stay valid while every particle is
// within its skin of its position at the build (tested exactly after every
// drift) and within R of its H; a pair then cannot come within range
// without being listed.  Work unit: a chunk, i.e. up to 64 particles of one
// leaf cell (one wave).  A chunk keeps the union U of its particles' lists
// (particle indices, in the order the cells were visited) and each particle
// keeps its own list as 16-bit positions in U, ascending.  The density sweeps
// and the force stage U once per chunk into LDS (coordinates relative to the
// chunk's first particle) and every lane then loops over its own list only:
// no candidate tests against whole cells and no per-pair global gathers.
//
// Positions of the list kernels are fixed-point integers per box axis,
// X = round(x / L 2^B) mod 2^B (B = 32 for the FP32 modes, 64 for FP64).
// The difference of two such integers is exact, wraps to the minimum
// periodic image by itself, and is converted to the compute precision only
// then: x_i - x_j = (int)(X_i - X_j) L 2^-B.  In the FP32 modes each
// coordinate also keeps its remainder r = x - X L 2^-32 (|r| <= L 2^-33) as
// a float, and x_i - x_j = (int)(X_i - X_j) L 2^-32 + (r_i - r_j): the pair
// offset is then as accurate as FP32 allows (relative 6e-8) at any distance,
// where the integers alone would round positions to L 2^-33 (a relative
// error of 1e-5 of H for H ~ 1e-5 L).
//
// Layout: chunk c owns U[uo[c] .. uo[c+1]) and the rows ro[c] .. ro[c+1]-1
// of 64 16-bit entries (its longest list rounded up to a multiple of 8);
// rows are grouped by 8 lane-major, entry k of lane l at 64 ro[c] + 512
// (k / 8) + 8 l + k % 8, so one 16-byte load gives a lane 8 entries and a
// wave's loads of a group are one contiguous kilobyte.  A count pass sizes U
// and the rows, an emission pass writes them.  plen[p] = length of particle
// p's list.  The particle itself is not listed: its density term is added
// directly and its force term is zero.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "sph_ctx.h"
#include "sph_device.h"

// ---------------------------------------------------------------------------
// Fixed-point positions
// ---------------------------------------------------------------------------
template <typename T> struct PQ;
template <> struct __align__(16) PQ<float> {
    uint32_t x, y, z;
    float m;
};
template <> struct __align__(16) PQ<double> {
    uint64_t x, y, z;
    double m;
};

__device__ inline uint32_t fix32(double x, double L)
{
    const double q = x / L;  // [0, 1) for a particle inside its box
    return (uint32_t)(uint64_t)(q * 4294967296.0 + 0.5);  // 2^32 wraps to 0: the same periodic point
}
__device__ inline uint64_t fix64(double x, double L)
{
    const double q = (x / L) * 4294967296.0;  // exact scaling by 2^32
    const double hi = floor(q);
    const double lo = (q - hi) * 4294967296.0;
    return ((uint64_t)(uint32_t)(int64_t)hi << 32) + (uint64_t)lo;
}

// remainder of x after its 32-bit fixed-point value (|r| <= L 2^-33)
__device__ inline float fix32_rem(double x, uint32_t X, double L)
{
    double v = x - (double)X * (L * 2.3283064365386963e-10);
    if (v > 0.5 * L) v -= L;  // X wrapped from 2^32 to 0
    return (float)v;
}

// Fixed-point position and mass of one particle; the FP32 modes also write
// the remainders to rem (x, y, z; w is left to the ghost, which stores 1/H).
__device__ inline void put_pq(PQ<float>* pq, float4* rem, int64_t i, double x, double y, double z, double m,
                              const DomainInfo& I)
{
    PQ<float> q;
    q.x = fix32(x, I.L[0]);
    q.y = fix32(y, I.L[1]);
    q.z = fix32(z, I.L[2]);
    q.m = (float)m;
    pq[i] = q;
    float* r = (float*)&rem[i];
    r[0] = fix32_rem(x, q.x, I.L[0]);
    r[1] = fix32_rem(y, q.y, I.L[1]);
    r[2] = fix32_rem(z, q.z, I.L[2]);
}
__device__ inline void put_pq(PQ<double>* pq, float4*, int64_t i, double x, double y, double z, double m,
                              const DomainInfo& I)
{
    PQ<double> q;
    q.x = fix64(x, I.L[0]);
    q.y = fix64(y, I.L[1]);
    q.z = fix64(z, I.L[2]);
    q.m = m;
    pq[i] = q;
}

// Position of a particle as the pair kernels read it.
template <typename T> struct PPos;
template <> struct PPos<float> {
    uint32_t x, y, z;
    float m;
    float4 r;  // remainders, w = 1/H (force stage)
};
template <> struct PPos<double> {
    uint64_t x, y, z;
    double m;
};
__device__ inline PPos<float> load_pos(const PQ<float>* pq, const float4* rem, uint32_t j)
{
    const uint4 a = *(const uint4*)&pq[j];
    PPos<float> p;
    p.x = a.x;
    p.y = a.y;
    p.z = a.z;
    p.m = __uint_as_float(a.w);
    p.r = rem[j];
    return p;
}
__device__ inline PPos<double> load_pos(const PQ<double>* pq, const float4*, uint32_t j)
{
    const PQ<double> a = pq[j];
    PPos<double> p;
    p.x = a.x;
    p.y = a.y;
    p.z = a.z;
    p.m = a.m;
    return p;
}

// x_i - x_j (minimum image) from the fixed-point coordinates
__device__ inline void pos_diff(const PPos<float>& a, const PPos<float>& b, float sx, float sy, float sz, float& dx,
                                float& dy, float& dz)
{
    dx = fmaf((float)(int32_t)(a.x - b.x), sx, a.r.x - b.r.x);
    dy = fmaf((float)(int32_t)(a.y - b.y), sy, a.r.y - b.r.y);
    dz = fmaf((float)(int32_t)(a.z - b.z), sz, a.r.z - b.r.z);
}
__device__ inline void pos_diff(const PPos<double>& a, const PPos<double>& b, double sx, double sy, double sz,
                                double& dx, double& dy, double& dz)
{
    dx = (double)(int64_t)(a.x - b.x) * sx;
    dy = (double)(int64_t)(a.y - b.y) * sy;
    dz = (double)(int64_t)(a.z - b.z) * sz;
}

// length of one fixed-point unit along each axis of a box
template <typename T> __device__ inline T fix_unit(double L);
template <> __device__ inline float fix_unit<float>(double L) { return (float)(L * 2.3283064365386963e-10); }
template <> __device__ inline double fix_unit<double>(double L) { return L * 5.421010862427522e-20; }


// ---------------------------------------------------------------------------
// List radii and skins.  For lists kept over T = rebuild_steps dt (the step
// length of the build's step; T = 0 for a build outside a step):
//   skin  s_i = 1.2 (T |v_i| + T^2 |a_i| / 2), the particle's own displacement
//              over T with a margin;
//   radius R_i = H_i (1 + SPH_PLIST_SKIN) g_i, g_i the growth of H over T that
//              the energy equation predicts (d ln H/dt = -du/dt / (3 (gamma-1) u)
//              for these equations), by 1.2 and at most SPH_PLIST_GROWTH_MAX.
// Pre-pass (final = 0): per-box largest R and s, which size the top cells so
// that they cover max R + 2 max s (every pair that can come within range
// before the next build then lies in neighbouring top cells).  Final pass
// (after the grid): R, s and the list extent E = R + s per particle; in a
// box too small for the full allowances (three top cells of max R + 2 max s
// per dimension) skins and growth are scaled by the box's fraction alpha,
// and R stays within the top-cell edge minus twice the box's largest skin.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_plist_ext(int64_t n, const double* __restrict__ H,
                                                   const double* __restrict__ vx, const double* __restrict__ vy,
                                                   const double* __restrict__ vz, const double* __restrict__ ax,
                                                   const double* __restrict__ ay, const double* __restrict__ az,
                                                   const double* __restrict__ u, const double* __restrict__ dudt,
                                                   const int32_t* __restrict__ dom, const DomainInfo* __restrict__ di,
                                                   double gm1, double tk, int final, T* R, T* skin, double* E,
                                                   unsigned long long* boxmax)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i0 < n;
    const int64_t i = in ? i0 : n - 1;
    const int d = dom ? dom[i] : 0;
    const double h = H[i];
    double g = 1.0 + SPH_PLIST_SKIN, sk = 0.0;
    if (tk > 0.0) {
        const double v = sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        const double acc = sqrt(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
        sk = 1.2 * (tk * v + 0.5 * tk * tk * acc);
        const double ui = u[i];
        if (ui > 0.0 && dudt[i] < 0.0) {
            const double e = fmin(-tk * dudt[i] / (3.0 * gm1 * ui), 1.0);
            g *= fmin(1.0 + 1.2 * (exp(e) - 1.0), SPH_PLIST_GROWTH_MAX);
        }
    }
    double r = h * g;
    if (!final) {
        // one atomic per wave when its particles share a box (one contiguous
        // Morton range per box: all but the waves at box boundaries)
        const int d0 = __shfl(d, 0);
        if (__ballot(d != d0) == 0ull) {
            for (int off = 32; off > 0; off >>= 1) {
                r = fmax(r, __shfl_xor(r, off));
                sk = fmax(sk, __shfl_xor(sk, off));
            }
            if ((threadIdx.x & 63) == 0) {
                atomicMax(&boxmax[2 * d], (unsigned long long)__double_as_longlong(r));
                if (sk > 0.0) atomicMax(&boxmax[2 * d + 1], (unsigned long long)__double_as_longlong(sk));
            }
        } else {
            atomicMax(&boxmax[2 * d], (unsigned long long)__double_as_longlong(r));
            if (sk > 0.0) atomicMax(&boxmax[2 * d + 1], (unsigned long long)__double_as_longlong(sk));
        }
        return;
    }
    if (!in) return;
    const DomainInfo& I = di[d];
    r = h * ((1.0 + SPH_PLIST_SKIN) + I.pl_alpha * (g - (1.0 + SPH_PLIST_SKIN)));
    sk = fmin(I.pl_alpha * sk, I.pl_smax);
    const double s0min = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]);
    r = fmax(h, fmin(r, s0min - 2.0 * I.pl_smax));
    T rt = (T)r, st = (T)sk;
    if ((double)rt < r) rt = nextafter(rt, (T)INFINITY);
    if ((double)st < sk) st = nextafter(st, (T)INFINITY);
    R[i] = rt;
    skin[i] = st;
    E[i] = (double)rt + (double)st;
}

// Fixed-point positions after the cell lists, also kept as the positions of
// the build.
template <typename T>
__global__ __launch_bounds__(256) void k_plist_prep(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ y, const double* __restrict__ z,
                                                    const double* __restrict__ m, const int32_t* __restrict__ dom,
                                                    const DomainInfo* __restrict__ di, PQ<T>* pq, PQ<T>* pq0,
                                                    float4* rem)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DomainInfo& I = di[dom ? dom[i] : 0];
    put_pq(pq, rem, i, x[i], y[i], z[i], m[i], I);
    pq0[i] = pq[i];
}

// |X - X0| along the three axes, from fixed-point positions (minimum image)
__device__ inline double fix_disp(const PQ<float>& a, const PQ<float>& b, const DomainInfo& I)
{
    const double dx = (double)(int32_t)(a.x - b.x) * (I.L[0] * 2.3283064365386963e-10);
    const double dy = (double)(int32_t)(a.y - b.y) * (I.L[1] * 2.3283064365386963e-10);
    const double dz = (double)(int32_t)(a.z - b.z) * (I.L[2] * 2.3283064365386963e-10);
    return sqrt(dx * dx + dy * dy + dz * dz);
}
__device__ inline double fix_disp(const PQ<double>& a, const PQ<double>& b, const DomainInfo& I)
{
    const double dx = (double)(int64_t)(a.x - b.x) * (I.L[0] * 5.421010862427522e-20);
    const double dy = (double)(int64_t)(a.y - b.y) * (I.L[1] * 5.421010862427522e-20);
    const double dz = (double)(int64_t)(a.z - b.z) * (I.L[2] * 5.421010862427522e-20);
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Refresh after a drift with kept lists: new fixed-point positions, and the
// validity test of every particle's list: its displacement since the build
// within its skin (plus the FP32 rounding of the fixed-point positions) and
// its H (the start of this step's iteration) within R_i.
template <typename T>
__global__ __launch_bounds__(256) void k_plist_refresh(int64_t n, const double* __restrict__ x,
                                                       const double* __restrict__ y, const double* __restrict__ z,
                                                       const double* __restrict__ m, const double* __restrict__ H,
                                                       const int32_t* __restrict__ dom,
                                                       const DomainInfo* __restrict__ di, const T* __restrict__ R,
                                                       const T* __restrict__ skin, const PQ<T>* __restrict__ pq0,
                                                       PQ<T>* pq, float4* rem, int* flags,
                                                       unsigned long long* counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool moved = false, grown = false;
    if (i < n) {
        const DomainInfo& I = di[dom ? dom[i] : 0];
        put_pq(pq, rem, i, x[i], y[i], z[i], m[i], I);
        const double units = (sizeof(T) == 4 ? 2.3283064365386963e-10 : 0.0) * fmax(fmax(I.L[0], I.L[1]), I.L[2]);
        moved = !(fix_disp(pq[i], pq0[i], I) + 2.0 * units <= (double)skin[i]);
        grown = !(H[i] <= (double)R[i]);
    }
    const unsigned long long bm = __ballot(moved), bg = __ballot(grown);
    if ((threadIdx.x & 63) == 0 && (bm | bg)) {
        atomicOr(flags, FLAG_STALE);
        if (bm) atomicAdd(&counters[CNT_STALE_MOVED], (unsigned long long)__popcll(bm));
        if (bg) atomicAdd(&counters[CNT_STALE_GROWN], (unsigned long long)__popcll(bg));
    }
}

// ---------------------------------------------------------------------------
// List build: one wave per leaf A, chunks of 64 of its particles.  The
// candidates of A's neighbour-cell list that pass the box test are packed in
// A's frame into LDS tiles of 64 (cell-relative coordinates); per tile,
// j-major ballots give each particle its 64-bit mask of candidates within
// max(R_i, R_j) + s_i + s_j (grown by a rounding margin); the union of the masks is the
// tile's contribution to U, and each lane appends the positions in U of its
// own set bits.  EMIT = false counts (|U| per chunk, list lengths), EMIT =
// true writes U and the lists at the offsets the counts gave.
// ---------------------------------------------------------------------------
#define PB_ENTRIES 32
#define PLIST_ROUND 2e-5  // relative margin of the build's FP32 range tests

struct PlistBuildArgs {
    int n_leaves;
    const int* l_begin;
    const int* l_count;
    const double* l_origin;
    const double* l_hlist;
    const double* l_lo;
    const double* l_hi;
    const int* l_dom;
    const int* l_off;
    const ListEntry* list;
    const DomainInfo* di;
    const void* pos4;  // leaf-relative positions, w = m
    const void* R;     // list radii
    const void* skin;  // skins
    double smax;       // largest skin
    const int* cb;     // first chunk of each leaf
    int* ch_p0;        // per chunk: first particle, particle count (count pass)
    int* ch_n;
    int* cu;           // count pass: |U| per chunk; emission: offsets uo
    int* cw;           // count pass: rows per chunk; emission: offsets ro
    int* plen;         // list length per particle
    uint32_t* U;       // emission pass
    uint16_t* L;
    int* flags;
    unsigned long long* n_entries;
};

template <typename T>
struct PBTile {
    typename vec4<T>::type cp[128];  // candidate in A's frame, w = R_j
    T cs[128];                       // candidate's skin
    int cj[128];                     // candidate particle index
    typename vec4<T>::type si[64];   // i of A: x, y, z (A frame), R_i (negative: no particle)
    T ss[64];                        // skin of i
    EBatchBox<T, PB_ENTRIES> e;
};

template <typename T, bool EMIT>
__device__ void plist_leaf(const PlistBuildArgs& a, int A, PBTile<T>& L, int lane)
{
    typedef typename vec4<T>::type V4;
    const V4* pos4 = (const V4*)a.pos4;
    const T* R = (const T*)a.R;
    const T* SK = (const T*)a.skin;
    const int bA = a.l_begin[A], nA = a.l_count[A];
    const double oA[3] = {a.l_origin[3 * A], a.l_origin[3 * A + 1], a.l_origin[3 * A + 2]};
    const DomainInfo& I = a.di[a.l_dom[A]];
    const int e0 = a.l_off[A], e1 = a.l_off[A + 1];
    const T big = T(1e30), grow = T(1) + T(PLIST_ROUND);
    const T smax = (T)a.smax;
    unsigned long long nent = 0;
    for (int c0 = 0; c0 < nA; c0 += 64) {
        const int ci = a.cb[A] + (c0 >> 6);
        const int nc = min(64, nA - c0);
        const bool vi = lane < nc;
        const int i = bA + c0 + (vi ? lane : 0);
        const unsigned long long vmask = __ballot(vi);
        const V4 pi = pos4[i];
        const T Ri = R[i], si = SK[i];
        int len = 0;       // entries of this lane's list so far
        int ubase = 0;     // size of the chunk's union so far (wave-uniform)
        int uo = 0, row0 = 0, width = 0;
        if (EMIT) {
            uo = a.cu[ci];
            row0 = a.cw[ci];
            width = a.cw[ci + 1] - row0;
        }
        const double hA = wave_max(vi ? (double)Ri : 0.0);
        const T sA = (T)wave_max(vi ? (double)si : 0.0);
        const T hAm = (T)(hA * (1.0 + 1e-5));
        const T bxl = wave_min_t<T>(vi ? pi.x : big), bxh = wave_max_t<T>(vi ? pi.x : -big);
        const T byl = wave_min_t<T>(vi ? pi.y : big), byh = wave_max_t<T>(vi ? pi.y : -big);
        const T bzl = wave_min_t<T>(vi ? pi.z : big), bzh = wave_max_t<T>(vi ? pi.z : -big);
        wave_sync();
        {
            V4 q = pi;
            q.w = vi ? Ri : T(-1);
            L.si[lane] = q;
            L.ss[lane] = si;
        }
        T tlo[3] = {big, big, big}, thi[3] = {-big, -big, -big};
        T thl = T(0);
        auto run_tile = [&](int ln) {
            wave_sync();
            const V4 pj = L.cp[lane];
            const T sj = L.cs[lane];
            const int jg = L.cj[lane];
            const bool lv = lane < ln;
            // the cells' list radii cover max(R_j) + 2 smax
            const T Rt = fmax(Ri + si + smax, thl) * T(1.00001);
            const unsigned long long imask =
                vmask & __ballot(box_d2<T>(pi.x, pi.y, pi.z, tlo[0], tlo[1], tlo[2], thi[0], thi[1], thi[2]) < Rt * Rt);
            int mlo = 0, mhi = 0;
            unsigned long long um = 0ull;
            for (unsigned long long m = imask; m; m &= m - 1ull) {
                const int ii = uniform(__ffsll((long long)m) - 1);
                const V4 q = L.si[ii];
                const T dx = pj.x - q.x, dy = pj.y - q.y, dz = pj.z - q.z;
                const T lim = fmax(q.w, pj.w) + L.ss[ii] + sj;
                const unsigned long long hm = __ballot(lv && dx * dx + dy * dy + dz * dz < lim * lim * grow);
                um |= hm;
                mlo = amdgcn_writelane((int)(uint32_t)hm, ii, mlo);
                mhi = amdgcn_writelane((int)(uint32_t)(hm >> 32), ii, mhi);
            }
            // candidates any particle of the chunk needs join U, in tile order
            if (EMIT && ((um >> lane) & 1ull) && ubase + mask_rank(um, lane) < 65536)
                a.U[uo + ubase + mask_rank(um, lane)] = (uint32_t)jg;
            if (vi) {
                unsigned long long m = ((unsigned long long)(uint32_t)mhi << 32) | (uint32_t)mlo;
                while (m) {
                    const int sl = __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    if (L.cj[sl] == i) continue;
                    // the emission pass repeats the count pass's decisions
                    // exactly; the bounds only guard the chunk's rows
                    if (EMIT && len < width)
                        a.L[(size_t)row0 * 64 + (size_t)(len >> 3) * 512 + lane * 8 + (len & 7)] =
                            (uint16_t)(ubase + mask_rank(um, sl));
                    len++;
                }
            }
            ubase += __popcll(um);
            wave_sync();
        };
        int ncand = 0;
        for (int eb = e0; eb < e1; eb += PB_ENTRIES) {
            const int nbt = min(PB_ENTRIES, e1 - eb);
            const double* hl = a.l_hlist;
            const int nv = load_batch_box<T>(a.list, eb, nbt, lane, a.l_begin, a.l_count, a.l_origin, a.l_lo, a.l_hi,
                                             hl, oA, I, 1e-5 * hA,
                                             [&](const ListEntry& E) { return E.dist < fmax(hA + 2.0 * a.smax, hl[E.B]); },
                                             L.e);
            for (int k = 0; k < nv; k++) {
                const int bB = L.e.b[k], nB = L.e.n[k];
                const T dox = L.e.ox[k], doy = L.e.oy[k], doz = L.e.oz[k];
                for (int p0 = 0; p0 < nB; p0 += 64) {
                    const int ln = min(64, nB - p0);
                    bool in = false;
                    V4 q;
                    T rj = T(0), sj = T(0);
                    if (lane < ln) {
                        q = pos4[bB + p0 + lane];
                        rj = R[bB + p0 + lane];
                        sj = SK[bB + p0 + lane];
                        q.x += dox;
                        q.y += doy;
                        q.z += doz;
                        const T Rj = (fmax(hAm, rj) + sA + sj) * T(1.00001);
                        in = box_d2<T>(q.x, q.y, q.z, bxl, byl, bzl, bxh, byh, bzh) < Rj * Rj;
                    }
                    const unsigned long long mk = __ballot(in);
                    if (in) {
                        const int slot = ncand + mask_rank(mk, lane);
                        q.w = rj;
                        L.cp[slot] = q;
                        L.cs[slot] = sj;
                        L.cj[slot] = bB + p0 + lane;
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
                        V4 t0;
                        T ts = T(0);
                        int t1 = 0;
                        if (lane < rest) {
                            t0 = L.cp[64 + lane];
                            ts = L.cs[64 + lane];
                            t1 = L.cj[64 + lane];
                        }
                        wave_sync();
                        if (lane < rest) {
                            L.cp[lane] = t0;
                            L.cs[lane] = ts;
                            L.cj[lane] = t1;
                        }
                        ncand = rest;
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
        if (!EMIT) {
            if (vi) {
                a.plen[i] = len;
                nent += (unsigned long long)len;
            }
            int wmax = vi ? len : 0;
            for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off));
            wmax = (wmax + 7) & ~7;  // whole groups of 8 rows
            if (lane == 0) {
                a.ch_p0[ci] = bA + c0;
                a.ch_n[ci] = nc;
                a.cu[ci] = ubase;
                a.cw[ci] = wmax;
                if (ubase > 65535) atomicOr(a.flags, FLAG_INVALID);  // positions in U are 16-bit
            }
        }
        wave_sync();
    }
    for (int off = 32; off > 0; off >>= 1) nent += __shfl_xor(nent, off);
    if (lane == 0 && nent) atomicAdd(a.n_entries, nent);
}

template <typename T, bool EMIT>
__global__ __launch_bounds__(256) void k_plist_build(PlistBuildArgs a)
{
    __shared__ PBTile<T> tiles[WAVES_PER_WG];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int A = uniform(xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_WG + w);
    if (A >= a.n_leaves) return;
    plist_leaf<T, EMIT>(a, A, tiles[w], lane);
}

// Chunks of each leaf: ceil(count / 64).
__global__ __launch_bounds__(256) void k_leaf_chunks(int n_leaves, const int* __restrict__ l_count, int* nch)
{
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A < n_leaves) nch[A] = (l_count[A] + 63) >> 6;
}

// ---------------------------------------------------------------------------
// Staged chunk kernels.  The chunk's union U is loaded in segments of TILE
// candidates into LDS, as coordinates relative to the chunk's first particle
// (the cell-relative frame: within the chunk's leaf, whose extent the build
// bounds by its smallest H) with the per-candidate data of the stage; each
// lane then evaluates the entries of its own list that fall in the segment.
// Frame offsets are minimum images; their difference is the pair's minimum
// image unless the offsets of the segment and of the chunk's particles can
// add up to half a box edge (boxes not much larger than the largest H), in
// which case the pair offsets are wrapped once more.
// ---------------------------------------------------------------------------

// Whether the pair offsets x_i - x_j of a segment need wrapping: the largest
// |offset| along each axis among the chunk's particles (mi) and among the
// staged candidates (mj) together reach half the box edge.
template <typename T>
__device__ inline bool seg_wrap(T mix, T miy, T miz, T mjx, T mjy, T mjz, const DomainInfo& I)
{
    mjx = wave_max_t<T>(mjx);
    mjy = wave_max_t<T>(mjy);
    mjz = wave_max_t<T>(mjz);
    return (double)(mix + mjx) >= 0.49 * I.L[0] || (double)(miy + mjy) >= 0.49 * I.L[1] ||
           (double)(miz + mjz) >= 0.49 * I.L[2];
}

template <typename T>
__device__ inline void wrap_pair(T& dx, T& dy, T& dz, T Lx, T Ly, T Lz)
{
    dx -= Lx * rint(dx / Lx);
    dy -= Ly * rint(dy / Ly);
    dz -= Lz * rint(dz / Lz);
}
struct ChunkArgs {
    int n_chunks;
    const int* nch_dev;  // graph mode: chunk count read on the device (NULL: n_chunks)
    const int* ch_p0;
    const int* ch_n;
    const int* uo;
    const int* ro;
    const uint32_t* U;
    const uint16_t* L;
    const int* plen;
    const void* pq;
    const float4* rem;
    const int32_t* dom;
    const DomainInfo* di;
};

template <typename T>
__device__ inline void frame_pos(const PPos<T>& X, const PPos<T>& F, T sx, T sy, T sz, T& x, T& y, T& z)
{
    pos_diff(X, F, sx, sy, sz, x, y, z);
}

// Entry k of a lane's list from its loaded group of 8 (16-bit positions in U).
__device__ inline int group_entry(const uint4& g, int k)
{
    const unsigned long long lo = ((unsigned long long)g.y << 32) | g.x;
    const unsigned long long hi = ((unsigned long long)g.w << 32) | g.z;
    return (int)(((k & 4) ? hi : lo) >> ((k & 3) * 16)) & 0xffff;
}

// Walk a lane's list: fn(e) for every entry e (a position in U) below `lim`,
// from entry k on; groups of 8 are loaded one ahead.  Returns the first entry
// not taken.  All entries are taken when lim >= |U|.
template <typename F>
__device__ inline int walk_list(const uint4* grp, int len, int k, int lim, F fn)
{
    if (k >= len) return k;
    uint4 cur = grp[(k >> 3) * 64];
    while (k < len) {
        const int g = k >> 3;
        const int gend = min(len, (g + 1) * 8);
        uint4 nxt = cur;
        if (gend < len) nxt = grp[(g + 1) * 64];
        bool stop = false;
        for (; k < gend; k++) {
            const int e = group_entry(cur, k & 7);
            if (e >= lim) {
                stop = true;
                break;
            }
            fn(e);
        }
        if (stop) break;
        cur = nxt;
    }
    return k;
}

// Stage members [seg, seg + ns) of the chunk's union: candidate t of lane l
// is t = l + 64 m; the union indices of a batch are loaded first, then their
// particle data, so the loads of a batch are in flight together.
#define STAGE_BATCH 4

// Density sweep over the chunk lists + FP64 Newton step (eq. (rho)).
struct DensChunkArgs {
    DensArgs d;
    ChunkArgs c;
    const void* R;
};

template <typename T, bool COMP, int TILE>
__global__ __launch_bounds__(64) void k_density_chunks(DensChunkArgs la)
{
    typedef typename vec4<T>::type V4;
    constexpr bool EXTRAP = sizeof(T) == 4;
    __shared__ V4 P[TILE];
    const DensArgs& a = la.d;
    const ChunkArgs& C = la.c;
    if (a.gate && uniform(*a.gate) != 0) return;
    const int nC = C.nch_dev ? uniform(*C.nch_dev) : C.n_chunks;
    const int c = uniform(xcd_block(blockIdx.x, gridDim.x));
    if (c >= nC) return;
    const int lane = threadIdx.x;
    const int p0 = C.ch_p0[c], nc = C.ch_n[c];
    const bool valid = lane < nc;
    const int i = p0 + (valid ? lane : 0);
    const bool act = valid && !a.conv[i];
    if (__ballot(act) == 0ull) return;
    const PQ<T>* pq = (const PQ<T>*)C.pq;
    const PPos<T> Xf = load_pos(pq, C.rem, (uint32_t)p0), Xi = load_pos(pq, C.rem, (uint32_t)i);
    const DomainInfo& I = C.di[C.dom ? C.dom[p0] : 0];
    const T sx = fix_unit<T>(I.L[0]), sy = fix_unit<T>(I.L[1]), sz = fix_unit<T>(I.L[2]);
    T xi, yi, zi;
    frame_pos(Xi, Xf, sx, sy, sz, xi, yi, zi);
    const T mix = wave_max_t<T>(fabs(xi)), miy = wave_max_t<T>(fabs(yi)), miz = wave_max_t<T>(fabs(zi));
    const T Lx = (T)I.L[0], Ly = (T)I.L[1], Lz = (T)I.L[2];
    bool wrap = false;
    const double Hd = a.H[i];
    const T Hi = (T)Hd, H2 = Hi * Hi, invH = T(1) / Hi;
    Acc<T, COMP> sw, sd;
    T s2 = T(0);
    int cnt = 1;
    // the particle itself: w(0) = 1, 3 w(0) + 0 w'(0) = 3, no second-derivative term
    sw.add(Xi.m);
    sd.add(T(3) * Xi.m);
    const int u0 = C.uo[c], nU = C.uo[c + 1] - u0;
    const int len = act ? C.plen[i] : 0;
    const uint4* grp = (const uint4*)(C.L + (size_t)C.ro[c] * 64) + lane;
    int k = 0;
    for (int seg = 0; seg < nU; seg += TILE) {
        const int ns = min(TILE, nU - seg);
        wave_sync();
        T mjx = T(0), mjy = T(0), mjz = T(0);
        for (int t0 = 0; t0 < ns; t0 += 64 * STAGE_BATCH) {
            uint32_t jb[STAGE_BATCH];
#pragma unroll
            for (int b = 0; b < STAGE_BATCH; b++) {
                const int t = t0 + b * 64 + lane;
                jb[b] = t < ns ? C.U[u0 + seg + t] : (uint32_t)p0;
            }
            PPos<T> Xb[STAGE_BATCH];
#pragma unroll
            for (int b = 0; b < STAGE_BATCH; b++) Xb[b] = load_pos(pq, C.rem, jb[b]);
#pragma unroll
            for (int b = 0; b < STAGE_BATCH; b++) {
                const int t = t0 + b * 64 + lane;
                if (t < ns) {
                    V4 q;
                    frame_pos(Xb[b], Xf, sx, sy, sz, q.x, q.y, q.z);
                    q.w = (T)Xb[b].m;
                    P[t] = q;
                    mjx = fmax(mjx, fabs(q.x));
                    mjy = fmax(mjy, fabs(q.y));
                    mjz = fmax(mjz, fabs(q.z));
                }
            }
        }
        wrap = seg_wrap(mix, miy, miz, mjx, mjy, mjz, I);
        wave_sync();
        k = walk_list(grp, len, k, seg + ns, [&](int e) {
            const V4 q = P[e - seg];
            T dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
            if (wrap) wrap_pair(dx, dy, dz, Lx, Ly, Lz);
            const T r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < H2) {
                const T qq = fast_sqrt(r2) * invH;
                T wv, dw;
                spline_w_dw(qq, wv, dw);
                sw.add(q.w * wv);
                sd.add(q.w * (T(3) * wv + qq * dw));
                if (EXTRAP) s2 += q.w * spline_d2(qq, dw);
                cnt++;
            }
        });
    }
    {
        unsigned long long ev = act ? (unsigned long long)cnt : 0ull;
        for (int off = 32; off > 0; off >>= 1) ev += __shfl_xor(ev, off);
        if (lane == 0 && ev) atomicAdd(&a.counters[CNT_DEVAL], ev);
    }
    bool left = false;
    if (act) {
        const double hlim = fmin(fmin(I.L[0], I.L[1]), I.L[2]) / 3.0;
        // the top cells cover the list radii plus twice the box's largest skin
        const double s0min = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]) - 2.0 * I.pl_smax;
        // the list holds every neighbour within R_i while the particles stay
        // within their skins (checked at every drift)
        const double hlA = (double)((const T*)la.R)[i];
        left = dens_newton<EXTRAP>(a, i, Hd, sw.total(), sd.total(), (double)s2, cnt, hlA, hlim, s0min);
    }
    const unsigned long long lm = __ballot(left);
    if (lm && lane == 0) atomicAdd(&a.counters[CNT_UNCONV], (unsigned long long)__popcll(lm));
}

// Force over the chunk lists, eqs. (dvdt) and (dudt): each particle sums its
// own pairs r < max(H_i, H_j) (every pair evaluated from both sides, no
// atomics).  From the ghost: fv4 = {v, A (8/pi) / H^4} and hf = 1/H.
struct ForceChunkArgs {
    ChunkArgs c;
    const void* fv4;
    const void* hf;
    double* ax;
    double* ay;
    double* az;
    double* dudt;
    int32_t* nngb;
    unsigned long long* counters;
    const int* gate;
};

template <typename T, bool COMP, int TILE>
__global__ __launch_bounds__(64) void k_force_chunks(ForceChunkArgs a)
{
    typedef typename vec4<T>::type V4;
    __shared__ V4 P[TILE];   // x, y, z (chunk frame), m
    __shared__ V4 V[TILE];   // vx, vy, vz, A (8/pi) / H^4
    __shared__ T IH[TILE];   // 1/H
    const ChunkArgs& C = a.c;
    if (a.gate && uniform(*a.gate) != 1) return;
    const int nC = C.nch_dev ? uniform(*C.nch_dev) : C.n_chunks;
    const int c = uniform(xcd_block(blockIdx.x, gridDim.x));
    if (c >= nC) return;
    const int lane = threadIdx.x;
    const int p0 = C.ch_p0[c], nc = C.ch_n[c];
    const bool valid = lane < nc;
    const int i = p0 + (valid ? lane : 0);
    const PQ<T>* pq = (const PQ<T>*)C.pq;
    const V4* fv4 = (const V4*)a.fv4;
    const T* hf = (const T*)a.hf;
    const PPos<T> Xf = load_pos(pq, C.rem, (uint32_t)p0), Xi = load_pos(pq, C.rem, (uint32_t)i);
    const DomainInfo& I = C.di[C.dom ? C.dom[p0] : 0];
    const T sx = fix_unit<T>(I.L[0]), sy = fix_unit<T>(I.L[1]), sz = fix_unit<T>(I.L[2]);
    T xi, yi, zi;
    frame_pos(Xi, Xf, sx, sy, sz, xi, yi, zi);
    const T mix = wave_max_t<T>(fabs(xi)), miy = wave_max_t<T>(fabs(yi)), miz = wave_max_t<T>(fabs(zi));
    const T Lx = (T)I.L[0], Ly = (T)I.L[1], Lz = (T)I.L[2];
    bool wrap = false;
    const V4 fi = fv4[i];
    const T ihi = hf[i];
    FAcc<T, COMP> ai;
    int nni = 1, nmax = 0;  // the particle itself counts within H_i
    const int u0 = C.uo[c], nU = C.uo[c + 1] - u0;
    const int len = valid ? C.plen[i] : 0;
    const uint4* grp = (const uint4*)(C.L + (size_t)C.ro[c] * 64) + lane;
    int k = 0;
    for (int seg = 0; seg < nU; seg += TILE) {
        const int ns = min(TILE, nU - seg);
        wave_sync();
        T mjx = T(0), mjy = T(0), mjz = T(0);
        for (int t0 = 0; t0 < ns; t0 += 64 * STAGE_BATCH) {
            uint32_t jb[STAGE_BATCH];
#pragma unroll
            for (int b = 0; b < STAGE_BATCH; b++) {
                const int t = t0 + b * 64 + lane;
                jb[b] = t < ns ? C.U[u0 + seg + t] : (uint32_t)p0;
            }
            PPos<T> Xb[STAGE_BATCH];
            V4 Fb[STAGE_BATCH];
            T Hb[STAGE_BATCH];
#pragma unroll
            for (int b = 0; b < STAGE_BATCH; b++) {
                Xb[b] = load_pos(pq, C.rem, jb[b]);
                Fb[b] = fv4[jb[b]];
                Hb[b] = hf[jb[b]];
            }
#pragma unroll
            for (int b = 0; b < STAGE_BATCH; b++) {
                const int t = t0 + b * 64 + lane;
                if (t < ns) {
                    V4 q;
                    frame_pos(Xb[b], Xf, sx, sy, sz, q.x, q.y, q.z);
                    q.w = (T)Xb[b].m;
                    P[t] = q;
                    V[t] = Fb[b];
                    IH[t] = Hb[b];
                    mjx = fmax(mjx, fabs(q.x));
                    mjy = fmax(mjy, fabs(q.y));
                    mjz = fmax(mjz, fabs(q.z));
                }
            }
        }
        wrap = seg_wrap(mix, miy, miz, mjx, mjy, mjz, I);
        wave_sync();
        k = walk_list(grp, len, k, seg + ns, [&](int e) {
            const V4 q = P[e - seg], fj = V[e - seg];
            const T ihj = IH[e - seg];
            T dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
            if (wrap) wrap_pair(dx, dy, dz, Lx, Ly, Lz);
            const T r2 = dx * dx + dy * dy + dz * dz;
            // coincident particles exert no force: at r2 = 0 the clamp gives
            // r = 0, dW/dr(0) = 0 and d = 0, so every term is an exact zero
            const T ir = fast_rsqrt(fmax(r2, T(1e-30)));
            const T r = r2 * ir;
            const T qi = r * ihi, qj = r * ihj;
            const T Fi = fi.w * spline_dw(qi);  // A_i dW/dr(r, H_i)
            const T Fj = fj.w * spline_dw(qj);  // A_j dW/dr(r, H_j)
            const T F = (Fi + Fj) * ir;
            const T dvdr = ((fi.x - fj.x) * dx + (fi.y - fj.y) * dy + (fi.z - fj.z) * dz) * ir;
            const T mjF = q.w * F;
            ai.ax.add(-mjF * dx);
            ai.ay.add(-mjF * dy);
            ai.az.add(-mjF * dz);
            ai.du.add(q.w * Fi * dvdr);
            nni += qi < T(1);
            nmax += (qi < T(1)) | (qj < T(1));
        });
    }
    unsigned long long np = 0, nd_w = 0;
    if (valid) {
        a.ax[i] = ai.ax.total();
        a.ay[i] = ai.ay.total();
        a.az[i] = ai.az.total();
        a.dudt[i] = ai.du.total();
        if (a.nngb) a.nngb[i] = nni;
        np = (unsigned long long)nmax;
        nd_w = (unsigned long long)nni;
    }
    for (int off = 32; off > 0; off >>= 1) {
        np += __shfl_xor(np, off);
        nd_w += __shfl_xor(nd_w, off);
    }
    if (lane == 0 && np) atomicAdd(&a.counters[CNT_NFORCE], np);
    if (lane == 0 && nd_w) atomicAdd(&a.counters[CNT_NDENS_F], nd_w);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

static sph_status read_ints(sph_ctx* c, const int* d, int* h, int n)
{
    SPH_CHECK_HIP(hipMemcpyAsync(h, d, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    return SPH_OK;
}

// Particle lists from the current cells, leaf lists and H (right after a
// cell build or a relist: no displacement since): chunks of the leaves,
// count pass, offsets, emission pass.
sph_status plist_build(sph_ctx* c)
{
    const int64_t n = c->n;
    const bool f64 = c->prm.precision == SPH_FP64;
    const size_t pqs = f64 ? sizeof(PQ<double>) : sizeof(PQ<float>);
    const int nL = c->n_leaves;
    SPH_TRY(buf_ensure(c->pq, (size_t)n * pqs));
    SPH_TRY(buf_ensure(c->plen, (size_t)n * sizeof(int)));
    SPH_TRY(buf_ensure(c->pq0, (size_t)n * pqs));
    if (!f64) SPH_TRY(buf_ensure(c->prem, (size_t)n * sizeof(float4)));
    const int nb = blocks_for(n, 256);
    if (f64)
        k_plist_prep<double><<<nb, 256, 0, c->stream>>>(n, c->P.x, c->P.y, c->P.z, c->P.m, c->P.domain,
                                                        (const DomainInfo*)c->dom_d.p, (PQ<double>*)c->pq.p,
                                                        (PQ<double>*)c->pq0.p, nullptr);
    else
        k_plist_prep<float><<<nb, 256, 0, c->stream>>>(n, c->P.x, c->P.y, c->P.z, c->P.m, c->P.domain,
                                                       (const DomainInfo*)c->dom_d.p, (PQ<float>*)c->pq.p,
                                                       (PQ<float>*)c->pq0.p, (float4*)c->prem.p);
    SPH_CHECK_LAUNCH();
    int* flags = (int*)c->flags.p;
    unsigned long long* cnt = (unsigned long long*)c->counters.p;
    // chunks: ceil(count / 64) per leaf
    SPH_TRY(buf_ensure(c->ch_base, (size_t)(nL + 1) * sizeof(int)));
    int* cb = (int*)c->ch_base.p;
    SPH_CHECK_HIP(hipMemsetAsync(cb + nL, 0, sizeof(int), c->stream));
    k_leaf_chunks<<<blocks_for(nL, 256), 256, 0, c->stream>>>(nL, (const int*)c->l_count.p, cb);
    SPH_CHECK_LAUNCH();
    SPH_TRY(scan_exclusive(c, cb, cb, nL + 1, flags + FI_PLROWS));
    int nC = 0;
    SPH_TRY(read_ints(c, flags + FI_PLROWS, &nC, 1));
    c->n_chunks = nC;
    SPH_TRY(buf_ensure(c->ch_p0, (size_t)(nC + 1) * sizeof(int)));
    SPH_TRY(buf_ensure(c->ch_n, (size_t)(nC + 1) * sizeof(int)));
    SPH_TRY(buf_ensure(c->ch_uo, (size_t)(nC + 1) * sizeof(int)));
    SPH_TRY(buf_ensure(c->ch_ro, (size_t)(nC + 1) * sizeof(int)));
    SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_NPLIST], 0, 8, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync((int*)c->ch_uo.p + nC, 0, sizeof(int), c->stream));
    SPH_CHECK_HIP(hipMemsetAsync((int*)c->ch_ro.p + nC, 0, sizeof(int), c->stream));
    PlistBuildArgs a;
    memset(&a, 0, sizeof(a));
    a.n_leaves = nL;
    a.l_begin = (const int*)c->l_begin.p;
    a.l_count = (const int*)c->l_count.p;
    a.l_origin = (const double*)c->l_origin.p;
    a.l_hlist = (const double*)c->l_hlist.p;
    a.l_lo = (const double*)c->l_lo.p;
    a.l_hi = (const double*)c->l_hi.p;
    a.l_dom = (const int*)c->l_dom.p;
    a.l_off = (const int*)c->l_off.p;
    a.list = (const ListEntry*)c->list.p;
    a.di = (const DomainInfo*)c->dom_d.p;
    a.pos4 = c->pos4.p;
    a.R = c->pR.p;
    a.skin = c->pskin.p;
    a.smax = c->skin_max;  // largest skin over the boxes
    a.cb = cb;
    a.ch_p0 = (int*)c->ch_p0.p;
    a.ch_n = (int*)c->ch_n.p;
    a.cu = (int*)c->ch_uo.p;
    a.cw = (int*)c->ch_ro.p;
    a.plen = (int*)c->plen.p;
    a.flags = flags;
    a.n_entries = &cnt[CNT_NPLIST];
    const int g = blocks_for(nL, WAVES_PER_WG);
    if (g > 0) {
        if (f64) k_plist_build<double, false><<<g, 256, 0, c->stream>>>(a);
        else k_plist_build<float, false><<<g, 256, 0, c->stream>>>(a);
        SPH_CHECK_LAUNCH();
    }
    // offsets of the unions and of the rows (totals behind them)
    SPH_TRY(scan_exclusive(c, (int*)c->ch_uo.p, (int*)c->ch_uo.p, nC + 1, flags + FI_PLROWS));
    SPH_TRY(scan_exclusive(c, (int*)c->ch_ro.p, (int*)c->ch_ro.p, nC + 1, flags + FI_SCRATCH));
    int tot[2] = {0, 0}, fl = 0;
    unsigned long long ne = 0;
    SPH_CHECK_HIP(hipMemcpyAsync(&tot[0], flags + FI_PLROWS, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(&tot[1], flags + FI_SCRATCH, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(&ne, &cnt[CNT_NPLIST], 8, hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    if (fl & FLAG_INVALID) return SPH_ERR_INVALID;  // a chunk's union exceeds 16-bit positions
    if (tot[0] < 0 || tot[1] < 0 || (int64_t)tot[1] * 64 > ((int64_t)1 << 40)) return SPH_ERR_WORKSPACE;
    c->n_union = tot[0];
    c->plist_rows = tot[1];
    c->n_plist = (int64_t)ne;
    SPH_TRY(buf_ensure(c->ch_U, (size_t)std::max(tot[0], 1) * sizeof(uint32_t)));
    SPH_TRY(buf_ensure(c->plist, (size_t)std::max(tot[1], 1) * 64 * sizeof(uint16_t)));
    a.cu = (int*)c->ch_uo.p;
    a.cw = (int*)c->ch_ro.p;
    a.U = (uint32_t*)c->ch_U.p;
    a.L = (uint16_t*)c->plist.p;
    if (g > 0) {
        if (f64) k_plist_build<double, true><<<g, 256, 0, c->stream>>>(a);
        else k_plist_build<float, true><<<g, 256, 0, c->stream>>>(a);
        SPH_CHECK_LAUNCH();
    }
    c->plist_valid = true;
    return SPH_OK;
}

// Per-box largest list radius and skin before the grid is chosen (out: 2 per
// box, as doubles), or the final radii, skins and extents of every particle.
sph_status plist_ext(sph_ctx* c, bool final, double* boxmax_host)
{
    const int64_t n = c->n;
    const int nd = c->prm.n_domains;
    const bool f64 = c->prm.precision == SPH_FP64;
    SPH_TRY(buf_ensure(c->pR, (size_t)n * (f64 ? 8 : 4)));
    SPH_TRY(buf_ensure(c->pskin, (size_t)n * (f64 ? 8 : 4)));
    SPH_TRY(buf_ensure(c->pext, (size_t)n * 8));
    SPH_TRY(buf_ensure(c->pbox, (size_t)nd * 16));
    if (!final) SPH_CHECK_HIP(hipMemsetAsync(c->pbox.p, 0, (size_t)nd * 16, c->stream));
    const double tk = c->prm.rebuild_steps > 0 ? c->prm.rebuild_steps * c->list_dt : 0.0;
    const int nb = blocks_for(n, 256);
    if (f64)
        k_plist_ext<double><<<nb, 256, 0, c->stream>>>(
            n, c->P.H, c->P.vx, c->P.vy, c->P.vz, c->P.ax, c->P.ay, c->P.az, c->P.u, c->P.dudt, c->P.domain,
            (const DomainInfo*)c->dom_d.p, c->prm.gamma - 1.0, tk, final ? 1 : 0, (double*)c->pR.p,
            (double*)c->pskin.p, (double*)c->pext.p, (unsigned long long*)c->pbox.p);
    else
        k_plist_ext<float><<<nb, 256, 0, c->stream>>>(
            n, c->P.H, c->P.vx, c->P.vy, c->P.vz, c->P.ax, c->P.ay, c->P.az, c->P.u, c->P.dudt, c->P.domain,
            (const DomainInfo*)c->dom_d.p, c->prm.gamma - 1.0, tk, final ? 1 : 0, (float*)c->pR.p,
            (float*)c->pskin.p, (double*)c->pext.p, (unsigned long long*)c->pbox.p);
    SPH_CHECK_LAUNCH();
    if (!final) {
        SPH_CHECK_HIP(hipMemcpyAsync(boxmax_host, c->pbox.p, (size_t)nd * 16, hipMemcpyDeviceToHost, c->stream));
        SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    }
    return SPH_OK;
}

// Kept lists after a drift: new fixed-point positions and the validity test
// (fresh = NULL: the flag and the counts stay on the device for the caller).
sph_status plist_refresh(sph_ctx* c, bool* fresh)
{
    int* flags = (int*)c->flags.p;
    unsigned long long* cnt = (unsigned long long*)c->counters.p;
    SPH_CHECK_HIP(hipMemsetAsync(flags, 0, sizeof(int), c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(&cnt[CNT_STALE_MOVED], 0, 16, c->stream));
    const int nb = blocks_for(c->n, 256);
    if (c->prm.precision == SPH_FP64)
        k_plist_refresh<double><<<nb, 256, 0, c->stream>>>(
            c->n, c->P.x, c->P.y, c->P.z, c->P.m, c->P.H, c->P.domain, (const DomainInfo*)c->dom_d.p,
            (const double*)c->pR.p, (const double*)c->pskin.p, (const PQ<double>*)c->pq0.p, (PQ<double>*)c->pq.p,
            nullptr, flags, cnt);
    else
        k_plist_refresh<float><<<nb, 256, 0, c->stream>>>(
            c->n, c->P.x, c->P.y, c->P.z, c->P.m, c->P.H, c->P.domain, (const DomainInfo*)c->dom_d.p,
            (const float*)c->pR.p, (const float*)c->pskin.p, (const PQ<float>*)c->pq0.p, (PQ<float>*)c->pq.p,
            (float4*)c->prem.p, flags, cnt);
    SPH_CHECK_LAUNCH();
    if (!fresh) return SPH_OK;  // the caller reads the flag and the counts
    int fl = 0;
    unsigned long long why[2] = {0, 0};
    SPH_CHECK_HIP(hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipMemcpyAsync(why, &cnt[CNT_STALE_MOVED], 16, hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    c->st.stale_moved = (int64_t)why[0];
    c->st.stale_grown = (int64_t)why[1];
    *fresh = !(fl & FLAG_STALE);
    return SPH_OK;
}

static void chunk_args(sph_ctx* c, bool graph, ChunkArgs& C)
{
    C.n_chunks = c->n_chunks;
    C.nch_dev = nullptr;
    (void)graph;
    C.ch_p0 = (const int*)c->ch_p0.p;
    C.ch_n = (const int*)c->ch_n.p;
    C.uo = (const int*)c->ch_uo.p;
    C.ro = (const int*)c->ch_ro.p;
    C.U = (const uint32_t*)c->ch_U.p;
    C.L = (const uint16_t*)c->plist.p;
    C.plen = (const int*)c->plen.p;
    C.pq = c->pq.p;
    C.rem = (const float4*)c->prem.p;
    C.dom = c->P.domain;
    C.di = (const DomainInfo*)c->dom_d.p;
}

// Segment sizes of the staged unions (an autotuner axis): density LDS holds
// TILE x 16 bytes (FP32), force TILE x 36 bytes.
template <typename T, bool COMP>
static void density_chunk_kernel(int tile, int nb, hipStream_t st, const DensChunkArgs& a)
{
    if (tile <= 256) k_density_chunks<T, COMP, 256><<<nb, 64, 0, st>>>(a);
    else if (tile <= 512) k_density_chunks<T, COMP, 512><<<nb, 64, 0, st>>>(a);
    else k_density_chunks<T, COMP, 1024><<<nb, 64, 0, st>>>(a);
}
template <typename T, bool COMP>
static void force_chunk_kernel(int tile, int nb, hipStream_t st, const ForceChunkArgs& a)
{
    if (tile <= 256) k_force_chunks<T, COMP, 256><<<nb, 64, 0, st>>>(a);
    else k_force_chunks<T, COMP, 512><<<nb, 64, 0, st>>>(a);
}

static int tile_or(int t, int dflt) { return t > 0 ? t : dflt; }

sph_status launch_density_plist(sph_ctx* c, const DensArgs& d)
{
    DensChunkArgs a;
    a.d = d;
    chunk_args(c, false, a.c);
    a.R = c->pR.p;
    const int nb = c->n_chunks;
    if (nb <= 0) return SPH_OK;
    const int tile = tile_or(c->prm.tile, c->prm.precision == SPH_FP64 ? 512 : 1024);
    if (c->prm.precision == SPH_FP64) density_chunk_kernel<double, false>(std::min(tile, 512), nb, c->stream, a);
    else if (c->prm.precision == SPH_FP32C) density_chunk_kernel<float, true>(tile, nb, c->stream, a);
    else density_chunk_kernel<float, false>(tile, nb, c->stream, a);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

sph_status launch_force_plist(sph_ctx* c, const int* gate)
{
    ForceChunkArgs a;
    memset(&a, 0, sizeof(a));
    chunk_args(c, false, a.c);
    a.fv4 = c->fv4.p;
    a.hf = c->hf.p;
    a.ax = c->P.ax;
    a.ay = c->P.ay;
    a.az = c->P.az;
    a.dudt = c->P.dudt;
    a.nngb = c->P.nngb;
    a.counters = (unsigned long long*)c->counters.p;
    a.gate = gate;
    const int nb = c->n_chunks;
    if (nb <= 0) return SPH_OK;
    const int tile = tile_or(c->prm.tile, 512);
    if (c->prm.precision == SPH_FP64) force_chunk_kernel<double, false>(std::min(tile, 256), nb, c->stream, a);
    else if (c->prm.precision == SPH_FP32C) force_chunk_kernel<float, true>(tile, nb, c->stream, a);
    else force_chunk_kernel<float, false>(tile, nb, c->stream, a);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}
