// Device-side helpers shared by the interaction kernels of libsph_hip
// (leaf-tile kernels and per-particle list kernels): the cubic-spline kernel
// of Sec. 2, compensated sums, wave reductions, the persistent task queues,
// pair-candidate batches of the neighbour-cell lists, and the density
// sweep's FP64 Newton step on rho H^3 = C.  Not part of the C-ABI.
#pragma once

#include <math.h>

#include "sph_ctx.h"

#define WAVES_PER_WG 4
#define INV_PI_8 2.5464790894703255  // 8/pi: cubic-spline normalisation in 3D

// ---------------------------------------------------------------------------
// Kernel shape, Sec. 2 (cubic spline with compact support H):
//   w(q)  = 1 - 6q^2 + 6q^3 (q <= 1/2),  2(1-q)^3 (1/2 < q < 1)
//   w'(q) = q(18q - 12)     (q <= 1/2), -6(1-q)^2 (1/2 < q < 1)
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void spline_w_dw(T q, T& w, T& dw)
{
    // both pieces and a select: lanes of a wave fall on both sides of q = 1/2
    const T t = T(1) - q;
    const bool in = q <= T(0.5);
    const T wi = T(1) + q * q * (T(6) * q - T(6)), dwi = q * (T(18) * q - T(12));
    const T wo = T(2) * t * t * t, dwo = T(-6) * t * t;
    w = in ? wi : wo;
    dw = in ? dwi : dwo;
}

// q^2 w''(q) + 2 q w'(q), the q-part of the second H-derivative of H^3 W
template <typename T>
__device__ inline T spline_d2(T q, T dw)
{
    const T di = T(36) * q - T(12), dout = T(12) * (T(1) - q);  // both pieces, then a select
    const T d2 = (q <= T(0.5)) ? di : dout;
    return q * (q * d2 + T(2) * dw);
}

template <typename T>
__device__ inline T spline_dw(T q)
{
    const T t = T(1) - q;
    const T vi = q * (T(18) * q - T(12)), vo = T(-6) * t * t;  // both pieces, then a select
    const T v = (q <= T(0.5)) ? vi : vo;
    return (q < T(1)) ? v : T(0);
}

// Square root, reciprocal square root and reciprocal: in FP32 the hardware
// instructions (1 ulp) instead of the longer correctly rounded sequences;
// FP64 keeps the IEEE operations.  Arguments are positive normal numbers.
__device__ inline float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fast_sqrt(double x) { return sqrt(x); }
__device__ inline float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double fast_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fast_rcp(double x) { return 1.0 / x; }

// Compensated (Kahan) accumulation; COMP = false gives the plain sum.
template <typename T, bool COMP>
struct Acc {
    T s = 0, c = 0;
    __device__ inline void add(T v)
    {
        if (COMP) {
            const T y = v - c;
            const T t = s + y;
            c = (t - s) - y;
            s = t;
        } else {
            s += v;
        }
    }
    __device__ inline double total() const { return COMP ? (double)s - (double)c : (double)s; }
};

__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}
__device__ inline float wave_minf(float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}
__device__ inline float wave_maxf(float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}
// Wave-uniform pop from a device task counter.  Every lane takes part in the
// atomic (lane 0 adds 1, the others 0) and the result is read from the first
// lane into a scalar register, so loops that exit on it have a uniform exit
// condition.  (A pop made by lane 0 alone inside `if (lane == 0)` lets the
// compiler treat the loop exit as divergent and run the other lanes on
// without lane 0.)
__device__ inline int wave_pop(unsigned long long* counter, int lane)
{
    const unsigned long long v = atomicAdd(counter, (unsigned long long)(lane == 0 ? 1 : 0));
    return __builtin_amdgcn_readfirstlane((int)v);
}

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Task queue of the persistent force kernels.  Task positions [0, nL) are cut into
// XQ_N = 8 contiguous ranges, one per XCD (workgroup b runs on XCD b mod 8),
// each drained through its own counter q[x * XQ_STRIDE].  A wave takes tasks
// from the range of its own XCD first, so the waves running side by side on
// one XCD work on neighbouring leaves and share its L2; once that range is
// empty it helps the other ranges in ring order, which balances ranges of
// unequal cost.  `k` (start at 0) is the number of ranges the wave has found
// empty; returns -1 when all are.  Every successful pop takes a distinct
// position, so a wave's loop over this ends after at most nL + 1 calls.
static_assert(XQ_N == 8, "one task range per XCD");
__device__ inline int xq_pop(unsigned long long* q, int nL, int& k, int lane)
{
    const int home = blockIdx.x & 7;
    while (k < XQ_N) {
        const int x = (home + k) & 7;
        const int lo = (int)(((long long)nL * x) >> 3), hi = (int)(((long long)nL * (x + 1)) >> 3);
        const long long t = (long long)lo + wave_pop(&q[x * XQ_STRIDE], lane);
        if (t < hi) return (int)t;
        k++;
    }
    return -1;
}

// v_writelane_b32: replace lane `lane` of `old` by the wave-uniform `src`
__device__ int amdgcn_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void shift_vec(int code, const DomainInfo& I, double* s)
{
    const int sh = code & 255;
    s[0] = (sh / 9 - 1) * I.L[0];
    s[1] = ((sh / 3) % 3 - 1) * I.L[1];
    s[2] = (sh % 3 - 1) * I.L[2];
}

// lanes per i-group for a chunk of nc particles: 8, 16, 32 or 64
__device__ inline int chunk_log2(int nc) { return nc <= 8 ? 3 : (nc <= 16 ? 4 : (nc <= 32 ? 5 : 6)); }

// Window [lo, hi) of B's particles (in the pair's sorted order) whose
// projection lies in [kmin, kmax).  Returns false if B is not sorted.
__device__ inline bool sorted_window(const float* skey, int64_t n, int dir, int bB, int nB, int lane, float kmin,
                                     float kmax, int& lo, int& hi)
{
    const float kb = (lane < nB) ? skey[(int64_t)dir * n + bB + lane] : INFINITY;
    lo = __popcll(__ballot(lane < nB && kb < kmin));
    hi = __popcll(__ballot(lane < nB && kb < kmax));
    return true;
}

// ---------------------------------------------------------------------------
// Pair-candidate selection.  For a neighbour cell B the particles that can
// interact with the wave's i particles are chosen either
//  - PRUNE_BOX: B's particles whose distance to the bounding box of the
//    wave's i particles is below the interaction range (3D test, one load of
//    B's cell per pair of cells, the next cell prefetched into registers), or
//  - PRUNE_SORTED: the window of B's particles sorted along the pair
//    direction whose projections lie within the range of the i projections
//    (the sort stage's per-direction order).
// ---------------------------------------------------------------------------
enum { PRUNE_BOX = 0, PRUNE_SORTED = 1 };

template <typename T> __device__ inline T wave_min_t(T v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}
template <typename T> __device__ inline T wave_max_t(T v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Squared distance from p to the box [lo, hi].
template <typename T>
__device__ inline T box_d2(T px, T py, T pz, T lx, T ly, T lz, T hx, T hy, T hz)
{
    const T gx = fmax(fmax(lx - px, px - hx), T(0));
    const T gy = fmax(fmax(ly - py, py - hy), T(0));
    const T gz = fmax(fmax(lz - pz, pz - hz), T(0));
    return gx * gx + gy * gy + gz * gz;
}

// lane position among the set lanes of mask below it
__device__ inline int mask_rank(unsigned long long mask, int lane)
{
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    return __popcll(mask & lt);
}

// Neighbour-entry batch of one wave, in LDS.
template <typename T, int NE = 64>
struct EBatch {
    int b[NE];     // first particle of B
    int n[NE];     // particles of B
    int B[NE];     // leaf index of B
    int dir[NE];   // sort direction of the pair
    T ox[NE], oy[NE], oz[NE];  // origin(B) + periodic shift - origin(A)
    T R[NE];       // interaction range of the pair (force)
};

// ---------------------------------------------------------------------------
// Density sweep + FP64 Newton step (eq. (rho); the smoothing-length
// constraint rho H^3 = C with its derivative 3 H^2 rho Omega).
// ---------------------------------------------------------------------------
struct DensArgs {
    int n_leaves;
    int64_t n;
    const int* l_begin;
    const int* l_count;
    const double* l_origin;
    const double* l_hlist;
    const double* l_lo;   // leaf boxes at the build (3 per leaf)
    const double* l_hi;
    const int* l_dom;
    const int* l_off;
    const ListEntry* list;
    int* l_active;
    const int* l_sorted;
    const void* pos4;
    const float* skey;
    const uint16_t* sidx;
    const DomainInfo* di;
    const double* m;
    double* H;
    double* rho;
    double* drho;
    double* hlo;
    double* hhi;
    uint8_t* conv;
    int32_t* nngb;
    double C_fac;
    double h_tol;
    int* flags;
    unsigned long long* counters;
    const double* margin;  // list margin: twice the largest displacement since the lists were built
    const int* gate;    // graph mode: skip the sweep unless *gate == 0 (NULL: always run)
    const int* nl_dev;  // graph mode: leaf count read from the device (NULL: n_leaves)
    int big_only;       // skip leaves of at most 64 particles (done by the packed kernel)
};

#define NTD 4  // neighbour cells per two-phase batch (density)

template <typename T>
struct DTile {
    typename vec4<T>::type p[NTD][64];  // selected particles of B (B frame), w = m
    EBatch<T> e;
};

// Load the entries [eb, eb + nbt) of A's list, keep those that pass
// keep(E), compact them into the batch; returns their number.
template <typename T, typename Keep, int NE = 64>
__device__ inline int load_batch(const ListEntry* list, int eb, int nbt, int lane, const int* l_begin, const int* l_count,
                                 const double* l_origin, const double* oA, const DomainInfo& I, Keep keep, EBatch<T, NE>& E,
                                 const double* l_hlist, int A)
{
    bool ok = false;
    ListEntry en;
    if (lane < nbt) {
        en = list[eb + lane];
        ok = keep(en);
    }
    const unsigned long long mask = __ballot(ok);
    if (ok) {
        const int s = mask_rank(mask, lane);
        const int B = en.B;
        double sv[3];
        shift_vec(en.code, I, sv);
        E.b[s] = l_begin[B];
        E.n[s] = l_count[B];
        E.B[s] = B;
        E.dir[s] = en.code >> 8;
        E.ox[s] = (T)(l_origin[3 * B] + sv[0] - oA[0]);
        E.oy[s] = (T)(l_origin[3 * B + 1] + sv[1] - oA[1]);
        E.oz[s] = (T)(l_origin[3 * B + 2] + sv[2] - oA[2]);
        E.R[s] = (T)(l_hlist ? l_hlist[B] : 0.0);
    }
    wave_sync();
    return __popcll(mask);
}

// FP64 Newton step of particle i after a sweep at H (Sec. 2: the constraint
// rho H^3 = C, whose H-derivative is 3 H^2 rho Omega): from the sums Sw =
// sum m_j w(q), Sd = sum m_j (3 w + q w') and, in the FP32 modes, S2 = sum
// m_j (q^2 w'' + 2 q w') (the second H-derivative of rho H^3 up to 8/pi /
// H^2), writes rho, d rho/dH and the count, tests |rho H^3 - C| <= tol C,
// and otherwise updates H inside the particle's bracket.  hlA: the largest H
// the particle's neighbour list covers (beyond it the list must be rebuilt);
// hlim: a third of the box edge; s0min: the smallest top-cell edge.
// Returns true if the particle is left unconverged.
template <bool EXTRAP>
__device__ inline bool dens_newton(const DensArgs& a, int i, double H, double Sw, double Sd, double S2, int cnt,
                                   double hlA, double hlim, double s0min)
{
    const double rho = INV_PI_8 / (H * H * H) * Sw;
    const double drho = -INV_PI_8 / (H * H * H * H) * Sd;
    const double C = a.C_fac * a.m[i];
    const double f = INV_PI_8 * Sw - C;              // rho H^3 - C
    const double fp = INV_PI_8 * (3.0 * Sw - Sd) / H; // 3 H^2 rho + H^3 drho/dH
    const double F2 = INV_PI_8 * S2 / (H * H);         // d^2 (rho H^3) / dH^2
    a.rho[i] = rho;
    a.drho[i] = drho;
    if (a.nngb) a.nngb[i] = cnt;
    bool left = false;
    bool done = fabs(f) <= a.h_tol * C;
    if (done && EXTRAP && f != 0.0) {
        // FP32 modes: the residual accepted here still moves rho by
        // f/C |1 - 1/Omega|; one Newton update of H with rho H^3 and its
        // H-derivative from their second-order expansion (as below) leaves
        // only the second-order term
        const double dH = -f / fp;
        const double Hn = H + dH;
        if (fabs(dH) <= 1e-3 * H && Hn <= hlA && Hn <= s0min) {
            const double F1 = INV_PI_8 * Sw + fp * dH + 0.5 * F2 * dH * dH;
            const double F1p = fp + F2 * dH;
            const double H3 = Hn * Hn * Hn;
            a.H[i] = Hn;
            a.rho[i] = F1 / H3;
            a.drho[i] = F1p / H3 - 3.0 * F1 / (H3 * Hn);
        }
    }
    if (!done) {
        double lo = a.hlo[i], hi = a.hhi[i];
        if (f < 0.0) lo = H;
        else hi = H;
        if (f < 0.0 && H >= hlim) {
            atomicOr(a.flags, FLAG_BOX_SMALL);
            done = true;
        } else {
            double Hn = H - f / fp;
            bool newton = true;
            if (!(Hn > lo && Hn < hi) || !isfinite(Hn)) {
                Hn = isinf(hi) ? 2.0 * H : 0.5 * (lo + hi);
                newton = false;
            }
            // at most doubling per sweep: a far-off step would only force
            // needless list and grid rebuilds before the bracket closes
            if (Hn > 2.0 * H) Hn = 2.0 * H;
            if (Hn > hlim) Hn = hlim;
            const double dH = Hn - H;
            if (fabs(dH) <= 4.0 * 2.220446049250313e-16 * H) {
                done = true;  // stalled at round-off: accept H
            } else if (EXTRAP && newton && fabs(dH) <= 1e-3 * H && Hn <= hlA && Hn <= s0min &&
                       fabs(0.5 * F2 * dH * dH) <= 0.5 * a.h_tol * C) {
                // accept the Newton update: rho H^3 and its H-derivative at Hn
                // from their second-order expansion around H
                const double F1 = INV_PI_8 * Sw + fp * dH + 0.5 * F2 * dH * dH;
                const double F1p = fp + F2 * dH;
                const double H3 = Hn * Hn * Hn;
                a.H[i] = Hn;
                a.rho[i] = F1 / H3;
                a.drho[i] = F1p / H3 - 3.0 * F1 / (H3 * Hn);
                done = true;
            } else {
                a.H[i] = Hn;
                a.hlo[i] = lo;
                a.hhi[i] = hi;
                if (Hn > hlA) atomicOr(a.flags, FLAG_RELIST);
                if (Hn > s0min) atomicOr(a.flags, FLAG_REBUILD);
                left = true;
            }
        }
    }
    if (done) {
        a.conv[i] = 1;
        atomicAdd(&a.counters[CNT_NDENS], (unsigned long long)cnt);
    }
    return left;
}

// Sums of one sweep -> rho, d rho/dH, neighbour count, and the FP64 Newton
// step (dens_newton).  The lanes of group 0 (jg == 0) own particle i; partial
// sums of the other groups are folded in first.  Returns true if particle i
// is left unconverged.
template <typename T>
__device__ inline bool dens_finish(const DensArgs& a, int i, bool act, int jg, int CI, double Hd, double Sw0,
                                   double Sd0, double S20, int cnt, double hlA, double hlim, double s0min)
{
    constexpr bool EXTRAP = sizeof(T) == 4;
    const int lane = threadIdx.x & 63;
    double Sw = Sw0, Sd = Sd0, S2 = S20;
    for (int off = CI; off < 64; off <<= 1) {
        Sw += __shfl_xor(Sw, off);
        Sd += __shfl_xor(Sd, off);
        if (EXTRAP) S2 += __shfl_xor(S2, off);
        cnt += __shfl_xor(cnt, off);
    }
    {
        // interactions evaluated by this sweep (lanes of group 0 hold the totals)
        unsigned long long ev = (jg == 0 && act) ? (unsigned long long)cnt : 0ull;
        for (int off = 32; off > 0; off >>= 1) ev += __shfl_xor(ev, off);
        if (lane == 0 && ev) atomicAdd(&a.counters[CNT_DEVAL], ev);
    }
    if (jg == 0 && act) return dens_newton<EXTRAP>(a, i, Hd, Sw, Sd, S2, cnt, hlA, hlim, s0min);
    return false;
}

// Neighbour-entry batch with each cell's box (at the build, A's frame,
// grown by `grow`), for the packed density path.
template <typename T, int NE>
struct EBatchBox {
    int b[NE], n[NE];
    T ox[NE], oy[NE], oz[NE];
    T lo[3][NE], hi[3][NE];
    T hl[NE];  // list radius of the cell (bounds its particles' H)
};

template <typename T, typename Keep, int NE>
__device__ inline int load_batch_box(const ListEntry* list, int eb, int nbt, int lane, const int* l_begin,
                                     const int* l_count, const double* l_origin, const double* l_lo, const double* l_hi,
                                     const double* l_hlist, const double* oA, const DomainInfo& I, double grow, Keep keep,
                                     EBatchBox<T, NE>& E)
{
    bool ok = false;
    ListEntry en;
    if (lane < nbt) {
        en = list[eb + lane];
        ok = keep(en);
    }
    const unsigned long long mask = __ballot(ok);
    if (ok) {
        const int s = mask_rank(mask, lane);
        const int B = en.B;
        double sv[3];
        shift_vec(en.code, I, sv);
        E.b[s] = l_begin[B];
        E.n[s] = l_count[B];
        E.ox[s] = (T)(l_origin[3 * B] + sv[0] - oA[0]);
        E.oy[s] = (T)(l_origin[3 * B + 1] + sv[1] - oA[1]);
        E.oz[s] = (T)(l_origin[3 * B + 2] + sv[2] - oA[2]);
        for (int d = 0; d < 3; d++) {
            E.lo[d][s] = (T)(l_lo[3 * B + d] + sv[d] - oA[d] - grow);
            E.hi[d][s] = (T)(l_hi[3 * B + d] + sv[d] - oA[d] + grow);
        }
        E.hl[s] = (T)l_hlist[B];
    }
    wave_sync();
    return __popcll(mask);
}

// Force sums of one particle (acceleration and du/dt).
template <typename T, bool COMP>
struct FAcc {
    Acc<T, COMP> ax, ay, az, du;
};

