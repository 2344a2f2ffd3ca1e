// SPH interpolation of a particle quantity at arbitrary points (paper,
// Sec. 2, eq. (interp)): Q(r) = sum_i m_i Q_i / rho_i W(|r - r_i|, H_i), each
// particle contributing within its own support H_i.
//
// The points are first ordered by box and Morton code of their position, so
// that the 64 points of a wave lie close together.  A wave whose points share
// a box and fit in a top cell (point sets dense against H) walks the octree of
// the last build once for all of them: cells farther from the wave's point box
// than their largest H are pruned, a leaf's particles are loaded one per lane
// and broadcast to the points with readlane, and only the particles that can
// reach the point box are visited.  Other waves (points sparse against H,
// several boxes, invalid points) walk the tree point by point, on nearby
// paths thanks to the order.
//
// Distances are minimum-image: every H is below half the box (the top cells
// are at least H wide and there are at least three per axis), so at most one
// image of a particle lies within its support.  Cell boxes are those of the
// build; particles have moved by at most delta since, so a cell is kept while
// its box lies closer than its largest H plus a margin of 2 delta.
#include <math.h>

#include "sph_ctx.h"

#define INTERP_INV_PI_8 2.5464790894703255  // 8/pi
#define INTERP_MBITS 10                    // Morton bits per axis of the sort key

namespace {

struct InterpArgs {
    int64_t m_pts;
    const double *px, *py, *pz;
    const int32_t* pdom;
    int n_dom;
    const DomainInfo* di;
    const Node* nodes;
    const WNode* wn;
    const double *x, *y, *z, *m, *rho, *H, *Q;
    double margin;
    double* out;
    const uint32_t* perm;  // sorted position -> point index
};

__device__ inline double interp_w(double q)
{
    if (!(q < 1.0)) return 0.0;
    return q <= 0.5 ? 1.0 + q * q * (6.0 * q - 6.0) : 2.0 * (1.0 - q) * (1.0 - q) * (1.0 - q);
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }

__device__ inline double wave_min_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}

__device__ inline double wave_max_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__device__ inline double readlane_d(double v, int l)
{
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Validated point k wrapped into its box; false for a bad box index or a
// non-finite coordinate.
__device__ inline bool load_point(const InterpArgs& a, int64_t k, double p[3], int& d)
{
    d = a.pdom ? a.pdom[k] : 0;
    p[0] = a.px[k];
    p[1] = a.py[k];
    p[2] = a.pz[k];
    if (d < 0 || d >= a.n_dom || !isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return false;
    const DomainInfo& I = a.di[d];
    for (int c = 0; c < 3; c++) {
        p[c] -= I.L[c] * floor(p[c] / I.L[c]);
        if (p[c] >= I.L[c]) p[c] = 0.0;  // a tiny negative input rounds up to L
    }
    return true;
}

// Top cells within reach of the box [lo, hi] (per axis: first cell and
// count, as residues of the periodic grid, each visited once).  Every H is at
// most the smallest top-cell edge once the density stage is done.
__device__ inline void top_range(const DomainInfo& I, const double lo[3], const double hi[3], double margin, int t0[3],
                                 int nt[3])
{
    const double R = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]) * (1.0 + 1e-9) + margin;
    for (int c = 0; c < 3; c++) {
        const int l = (int)floor((lo[c] - R) / I.s0[c]), h = (int)floor((hi[c] + R) / I.s0[c]);
        nt[c] = min(h - l + 1, I.n_top[c]);
        t0[c] = nt[c] == I.n_top[c] ? 0 : l;
    }
}

__device__ inline int top_index(const DomainInfo& I, const int t0[3], int ix, int iy, int iz)
{
    int c[3] = {t0[0] + ix, t0[1] + iy, t0[2] + iz};
    for (int q = 0; q < 3; q++) c[q] = ((c[q] % I.n_top[q]) + I.n_top[q]) % I.n_top[q];
    return I.top_offset + (c[0] * I.n_top[1] + c[1]) * I.n_top[2] + c[2];
}

// Squared minimum-image gap between a node's box and the box of centre c,
// half-widths hw.
__device__ inline double node_gap2(const Node& nd, const DomainInfo& I, const double c[3], const double hw[3])
{
    double d2 = 0.0;
    for (int q = 0; q < 3; q++) {
        const double half = 0.5 * (nd.hi[q] - nd.lo[q]);
        const double g = fmax(fabs(min_image(c[q] - 0.5 * (nd.lo[q] + nd.hi[q]), I.L[q])) - half - hw[q], 0.0);
        d2 += g * g;
    }
    return d2;
}

// One point, its own walk.
__device__ double interp_point(const InterpArgs& a, const DomainInfo& I, const double p[3])
{
    int t0[3], nt[3];
    top_range(I, p, p, a.margin, t0, nt);
    const double hw[3] = {0.0, 0.0, 0.0};
    double sum = 0.0;
    for (int ix = 0; ix < nt[0]; ix++)
    for (int iy = 0; iy < nt[1]; iy++)
    for (int iz = 0; iz < nt[2]; iz++) {
        int kk = top_index(I, t0, ix, iy, iz);
        while (kk >= 0) {
            const WNode w = a.wn[kk];
            if (w.count == 0) {
                kk = w.next;
                continue;
            }
            const Node& nd = a.nodes[kk];
            const double reach = nd.hmax + a.margin;
            if (node_gap2(nd, I, p, hw) >= reach * reach) {
                kk = w.next;
                continue;
            }
            if (w.first_child >= 0) {
                kk = w.first_child;
                continue;
            }
            kk = w.next;
            for (int i = nd.begin; i < nd.begin + nd.count; i++) {
                const double dx = min_image(p[0] - a.x[i], I.L[0]);
                const double dy = min_image(p[1] - a.y[i], I.L[1]);
                const double dz = min_image(p[2] - a.z[i], I.L[2]);
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                const double h = a.H[i];
                if (r < h) sum += a.m[i] * a.Q[i] / a.rho[i] * INTERP_INV_PI_8 / (h * h * h) * interp_w(r / h);
            }
        }
    }
    return sum;
}

// Sort keys: box index in the high bits, Morton code of the position
// (INTERP_MBITS per axis) below; invalid points get the largest key.
__global__ __launch_bounds__(256) void k_interp_keys(InterpArgs a, uint64_t* keys, uint32_t* vals, uint64_t invalid)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m_pts) return;
    double p[3];
    int d;
    uint64_t key = invalid;
    if (load_point(a, k, p, d)) {
        const DomainInfo& I = a.di[d];
        uint32_t f[3];
        for (int c = 0; c < 3; c++) {
            const double u = p[c] / I.L[c] * (1 << INTERP_MBITS);
            f[c] = (uint32_t)fmin(fmax(u, 0.0), (double)((1 << INTERP_MBITS) - 1));
        }
        uint64_t mort = 0;
        for (int b = INTERP_MBITS - 1; b >= 0; b--)
            mort = (mort << 3) | (((f[0] >> b) & 1u) << 2) | (((f[1] >> b) & 1u) << 1) | ((f[2] >> b) & 1u);
        key = ((uint64_t)d << (3 * INTERP_MBITS)) | mort;
    }
    keys[k] = key;
    vals[k] = (uint32_t)k;
}

// One wave per 64 consecutive points of the sorted order.
__global__ __launch_bounds__(256) void k_interp_wave(InterpArgs a)
{
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w * 64 >= a.m_pts) return;
    const int64_t s = w * 64 + lane;
    const bool inr = s < a.m_pts;
    const int64_t k = inr ? (int64_t)a.perm[s] : 0;
    double p[3] = {0.0, 0.0, 0.0};
    int d = -1;
    const bool ok = inr && load_point(a, k, p, d);
    if (inr && !ok) a.out[k] = NAN;
    const unsigned long long okm = __ballot(ok);
    if (okm == 0ull) return;
    const int d0 = __builtin_amdgcn_readlane(d, __ffsll((long long)okm) - 1);
    const DomainInfo& I = a.di[d0];
    const double big = 1e300;
    double lo[3], hi[3], c[3], hw[3];
    double ext = 0.0;
    for (int q = 0; q < 3; q++) {
        lo[q] = wave_min_d(ok ? p[q] : big);
        hi[q] = wave_max_d(ok ? p[q] : -big);
        c[q] = 0.5 * (lo[q] + hi[q]);
        hw[q] = 0.5 * (hi[q] - lo[q]);
        ext = fmax(ext, hi[q] - lo[q]);
    }
    const double s0min = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]);
    if (__ballot(ok && d != d0) != 0ull || !(ext <= s0min)) {
        if (ok) a.out[k] = interp_point(a, a.di[d], p);
        return;
    }
    int t0[3], nt[3];
    top_range(I, lo, hi, a.margin, t0, nt);
    double sum = 0.0;
    for (int ix = 0; ix < nt[0]; ix++)
    for (int iy = 0; iy < nt[1]; iy++)
    for (int iz = 0; iz < nt[2]; iz++) {
        int kk = __builtin_amdgcn_readfirstlane(top_index(I, t0, ix, iy, iz));
        while (kk >= 0) {
            const WNode wv = a.wn[kk];
            if (wv.count == 0) {
                kk = __builtin_amdgcn_readfirstlane(wv.next);
                continue;
            }
            const Node& nd = a.nodes[kk];
            const double reach = nd.hmax + a.margin;
            if (node_gap2(nd, I, c, hw) >= reach * reach) {
                kk = __builtin_amdgcn_readfirstlane(wv.next);
                continue;
            }
            if (wv.first_child >= 0) {
                kk = __builtin_amdgcn_readfirstlane(wv.first_child);
                continue;
            }
            kk = __builtin_amdgcn_readfirstlane(wv.next);
            const int b = nd.begin, n = nd.count;
            for (int p0 = 0; p0 < n; p0 += 64) {
                const bool has = p0 + lane < n;
                const int j = b + p0 + (has ? lane : 0);
                // the particle's image nearest the point box, its gap to that box
                double xj[3], g2 = 0.0;
                const double hj = a.H[j];
                {
                    const double r[3] = {a.x[j], a.y[j], a.z[j]};
                    for (int q = 0; q < 3; q++) {
                        xj[q] = c[q] + min_image(r[q] - c[q], I.L[q]);
                        const double g = fmax(fabs(xj[q] - c[q]) - hw[q], 0.0);
                        g2 += g * g;
                    }
                }
                const double cf = has ? a.m[j] * a.Q[j] / a.rho[j] * INTERP_INV_PI_8 / (hj * hj * hj) : 0.0;
                const double ih = 1.0 / hj, h2 = hj * hj;
                for (unsigned long long mk = __ballot(has && g2 < h2); mk; mk &= mk - 1ull) {
                    const int l = __ffsll((long long)mk) - 1;
                    const double jx = readlane_d(xj[0], l), jy = readlane_d(xj[1], l), jz = readlane_d(xj[2], l);
                    const double jh2 = readlane_d(h2, l);
                    const double dx = p[0] - jx, dy = p[1] - jy, dz = p[2] - jz;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (ok && r2 < jh2) sum += readlane_d(cf, l) * interp_w(sqrt(r2) * readlane_d(ih, l));
                }
            }
        }
    }
    if (ok) a.out[k] = sum;
}

}  // namespace

extern "C" sph_status sph_interpolate(sph_ctx* c, const double* Q, const double* px, const double* py,
                                      const double* pz, const int32_t* pdom, int64_t m_pts, double* out)
{
    if (!c || m_pts < 0 || ((!Q || !px || !py || !pz || !out) && m_pts > 0)) return SPH_ERR_INVALID;
    if (c->prm.n_domains > 1 && !pdom && m_pts > 0) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->dens_done) return SPH_ERR_STATE;
    if (m_pts == 0) return SPH_OK;
    if (m_pts > INT32_MAX) return SPH_ERR_INVALID;
    // largest H per cell from the current H (the lists keep their radii)
    SPH_TRY(node_hmax_all(c, false));
    InterpArgs a;
    a.m_pts = m_pts;
    a.px = px;
    a.py = py;
    a.pz = pz;
    a.pdom = pdom;
    a.n_dom = c->prm.n_domains;
    a.di = (const DomainInfo*)c->dom_d.p;
    a.nodes = (const Node*)c->nodes.p;
    a.wn = (const WNode*)c->wnodes.p;
    a.x = c->P.x;
    a.y = c->P.y;
    a.z = c->P.z;
    a.m = c->P.m;
    a.rho = c->P.rho;
    a.H = c->P.H;
    a.Q = Q;
    a.margin = 2.0 * c->delta;
    a.out = out;
    a.perm = nullptr;
    // sort the points by box and Morton code
    int dom_bits = 1;
    while ((1ll << dom_bits) <= (long long)c->prm.n_domains) dom_bits++;
    const int bits = dom_bits + 3 * INTERP_MBITS;
    for (int q = 0; q < 2; q++) {
        SPH_TRY(buf_ensure(c->ikeys[q], (size_t)m_pts * 8));
        SPH_TRY(buf_ensure(c->ivals[q], (size_t)m_pts * 4));
    }
    const unsigned nb = (unsigned)((m_pts + 255) / 256);
    k_interp_keys<<<nb, 256, 0, c->stream>>>(a, (uint64_t*)c->ikeys[0].p, (uint32_t*)c->ivals[0].p,
                                             (uint64_t)c->prm.n_domains << (3 * INTERP_MBITS));
    SPH_CHECK_LAUNCH();
    int res = 0;
    SPH_TRY(radix_sort(c, (int)m_pts, bits, c->ikeys, c->ivals, &res));
    a.perm = (const uint32_t*)c->ivals[res].p;
    const unsigned nw = (unsigned)((m_pts + 255) / 256);  // four waves of 64 points per workgroup
    k_interp_wave<<<nw, 256, 0, c->stream>>>(a);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}
