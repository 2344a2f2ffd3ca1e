// SPH interpolation of a particle quantity at arbitrary points (paper,
// Sec. 2, eq. (interp)): Q(r) = sum_i m_i Q_i / rho_i W(|r - r_i|, H_i), each
// particle contributing within its own support H_i.  One thread per point
// walks the octree of the last build from the top cells that can hold a
// contributing particle, pruning cells farther than their largest H.
//
// Distances are minimum-image: every H is below half the box (the top cells
// are at least H wide and there are at least three per axis), so at most one
// image of a particle lies within its support.  Cell boxes are those of the
// build; particles have moved by at most delta since, so a cell is kept while
// its box lies closer than its largest H plus a margin of 2 delta.
#include <math.h>

#include "sph_ctx.h"

#define INTERP_INV_PI_8 2.5464790894703255  // 8/pi

__device__ inline double interp_w(double q)
{
    if (!(q < 1.0)) return 0.0;
    return q <= 0.5 ? 1.0 + q * q * (6.0 * q - 6.0) : 2.0 * (1.0 - q) * (1.0 - q) * (1.0 - q);
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }

__global__ __launch_bounds__(256) void k_interp(int64_t m_pts, const double* __restrict__ px,
                                                const double* __restrict__ py, const double* __restrict__ pz,
                                                const int32_t* __restrict__ pdom, int n_dom,
                                                const DomainInfo* __restrict__ di,
                                                const Node* __restrict__ nodes, const WNode* __restrict__ wn,
                                                const double* __restrict__ x, const double* __restrict__ y,
                                                const double* __restrict__ z, const double* __restrict__ m,
                                                const double* __restrict__ rho, const double* __restrict__ H,
                                                const double* __restrict__ Q, double margin, double* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m_pts) return;
    const int d = pdom ? pdom[k] : 0;
    double p[3] = {px[k], py[k], pz[k]};
    if (d < 0 || d >= n_dom || !isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) {
        out[k] = NAN;
        return;
    }
    const DomainInfo& I = di[d];
    // top cells within (largest H + margin) of the point, as residues: every
    // H is at most the smallest top-cell edge once the density stage is done
    const double R = fmin(fmin(I.s0[0], I.s0[1]), I.s0[2]) * (1.0 + 1e-9) + margin;
    int t0[3], nt[3];
    for (int a = 0; a < 3; a++) {
        p[a] -= I.L[a] * floor(p[a] / I.L[a]);
        const int lo = (int)floor((p[a] - R) / I.s0[a]), hi = (int)floor((p[a] + R) / I.s0[a]);
        nt[a] = min(hi - lo + 1, I.n_top[a]);
        t0[a] = nt[a] == I.n_top[a] ? 0 : lo;
    }
    double sum = 0.0;
    for (int ix = 0; ix < nt[0]; ix++)
    for (int iy = 0; iy < nt[1]; iy++)
    for (int iz = 0; iz < nt[2]; iz++) {
        int c[3] = {t0[0] + ix, t0[1] + iy, t0[2] + iz};
        for (int a = 0; a < 3; a++) c[a] = ((c[a] % I.n_top[a]) + I.n_top[a]) % I.n_top[a];
        int kk = I.top_offset + (c[0] * I.n_top[1] + c[1]) * I.n_top[2] + c[2];
        while (kk >= 0) {
            const WNode w = wn[kk];
            if (w.count == 0) {
                kk = w.next;
                continue;
            }
            const Node& nd = nodes[kk];
            double d2 = 0.0;
            for (int a = 0; a < 3; a++) {
                const double half = 0.5 * (nd.hi[a] - nd.lo[a]);
                const double g = fmax(fabs(min_image(p[a] - 0.5 * (nd.lo[a] + nd.hi[a]), I.L[a])) - half, 0.0);
                d2 += g * g;
            }
            const double reach = nd.hmax + margin;
            if (d2 >= reach * reach) {
                kk = w.next;
                continue;
            }
            if (w.first_child >= 0) {
                kk = w.first_child;
                continue;
            }
            kk = w.next;
            for (int i = nd.begin; i < nd.begin + nd.count; i++) {
                const double dx = min_image(p[0] - x[i], I.L[0]);
                const double dy = min_image(p[1] - y[i], I.L[1]);
                const double dz = min_image(p[2] - z[i], I.L[2]);
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                const double h = H[i];
                if (r < h) sum += m[i] * Q[i] / rho[i] * INTERP_INV_PI_8 / (h * h * h) * interp_w(r / h);
            }
        }
    }
    out[k] = sum;
}

extern "C" sph_status sph_interpolate(sph_ctx* c, const double* Q, const double* px, const double* py,
                                      const double* pz, const int32_t* pdom, int64_t m_pts, double* out)
{
    if (!c || m_pts < 0 || ((!Q || !px || !py || !pz || !out) && m_pts > 0)) return SPH_ERR_INVALID;
    if (c->prm.n_domains > 1 && !pdom && m_pts > 0) return SPH_ERR_INVALID;
    if (!c->dens_done) return SPH_ERR_STATE;
    if (m_pts == 0) return SPH_OK;
    if (m_pts > INT32_MAX) return SPH_ERR_INVALID;
    // largest H per cell from the current H (the lists keep their radii)
    SPH_TRY(node_hmax_all(c, false));
    k_interp<<<(unsigned)((m_pts + 255) / 256), 256, 0, c->stream>>>(
        m_pts, px, py, pz, pdom, c->prm.n_domains, (const DomainInfo*)c->dom_d.p, (const Node*)c->nodes.p, (const WNode*)c->wnodes.p,
        c->P.x, c->P.y, c->P.z, c->P.m, c->P.rho, c->P.H, Q, 2.0 * c->delta, out);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}
