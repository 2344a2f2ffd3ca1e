// Learned smoothing-length predictor: per-particle features, the network's
// inference on the MFMA units, float32 training kernels (forward, backward,
// Adam) and the recording of training samples during steps.
//
// The predictor only moves the starting point of the Newton-Raphson solve of
// rho H^3 = (kernel_gamma eta)^3 m (paper, Sec. 2); the density sweeps still
// decide convergence.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "sph_ctx.h"

namespace {

constexpr int NIN = SPH_MLP_NIN, NH = SPH_MLP_NH, NT = SPH_MLP_NT, NP = SPH_MLP_NP, XS = SPH_MLP_XSTRIDE;
constexpr int O_W1 = 0, O_B1 = O_W1 + NIN * NH, O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH, O_W3 = O_B2 + NH,
              O_B3 = O_W3 + NH * NH, O_W4 = O_B3 + NH, O_B4 = O_W4 + NH, O_XMU = O_B4 + 1, O_XSD = O_XMU + NIN,
              O_YMU = O_XSD + NIN, O_YSD = O_YMU + 1;
static_assert(O_XMU == NT, "trained block");
static_assert(O_YSD + 1 == NP, "parameter vector");

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

// bfloat16: the top 16 bits of a float32, rounded to nearest, ties to even
__host__ __device__ inline uint16_t bf16_bits(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_float(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}
__device__ inline float bf16r(float x) { return bf16_float(bf16_bits(x)); }

__device__ inline float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float dsilu_f(float z)
{
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Inference weights arranged for v_mfma_f32_16x16x16_bf16.  The layers are
// computed transposed, Z^T = W^T X^T: A = a 16x16 block of W^T (output units
// x inputs), B = 16 inputs x 16 particles, D = 16 output units x 16
// particles.  Lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and
// D[4(l/16)+j][l%16] (j = 0..3), so the D block of output tile t is, after
// bias and SiLU, exactly the B operand of input chunk t of the next layer.
struct MlpPacked {
    bf16x4 a1[4][64];        // layer 1: [output tile][lane] (one input chunk)
    bf16x4 a2[4][4][64];     // layer 2: [output tile][input chunk][lane]
    bf16x4 a3[4][4][64];
    float b1[NH], b2[NH], b3[NH], w4[NH];
    float xmu[NIN], rxsd[NIN];
    float b4, ymu, ysd, pad;
};

}  // namespace

// ---------------------------------------------------------------------------
// Packing of the float32 parameter vector into the inference layout.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ p, MlpPacked* __restrict__ w)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // A operands: (layer, tile, chunk, lane) -> 4 weights
    const int n1 = 4 * 64, n2 = 16 * 64;
    if (t < n1 + 2 * n2) {
        int layer, tile, kc, lane;
        if (t < n1) {
            layer = 1;
            tile = t / 64;
            kc = 0;
            lane = t % 64;
        } else {
            const int r = (t - n1) % n2;
            layer = t < n1 + n2 ? 2 : 3;
            tile = r / 256;
            kc = (r / 64) % 4;
            lane = r % 64;
        }
        const float* W = layer == 1 ? p + O_W1 : layer == 2 ? p + O_W2 : p + O_W3;
        bf16x4 v;
        for (int j = 0; j < 4; j++) {
            const int k = kc * 16 + 4 * (lane / 16) + j;   // input unit
            const int o = tile * 16 + lane % 16;           // output unit
            v[j] = (short)bf16_bits(W[k * NH + o]);
        }
        if (layer == 1) w->a1[tile][lane] = v;
        else if (layer == 2) w->a2[tile][kc][lane] = v;
        else w->a3[tile][kc][lane] = v;
    }
    if (t < NH) {
        w->b1[t] = p[O_B1 + t];
        w->b2[t] = p[O_B2 + t];
        w->b3[t] = p[O_B3 + t];
        w->w4[t] = bf16_float(bf16_bits(p[O_W4 + t]));
    }
    if (t < NIN) {
        w->xmu[t] = p[O_XMU + t];
        w->rxsd[t] = 1.0f / p[O_XSD + t];
    }
    if (t == 0) {
        w->b4 = p[O_B4];
        w->ymu = p[O_YMU];
        w->ysd = p[O_YSD];
        w->pad = 0.f;
    }
}

// split x = hi + lo, both bfloat16 (hardware conversion, nearest even), for
// the four values of an operand
__device__ inline void split4(const float v[4], bf16x4& hi, bf16x4& lo)
{
    for (int j = 0; j < 4; j++) {
        const __bf16 h = (__bf16)v[j];
        const __bf16 l = (__bf16)(v[j] - (float)h);
        hi[j] = __builtin_bit_cast(short, h);
        lo[j] = __builtin_bit_cast(short, l);
    }
}

#define MFMA16(a, b, c) __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0)

// Network inference, one wave per 16 particles at a time.  Writes y (if
// non-NULL) and, if H is non-NULL, H[i] = H[i] exp(clamp(y, -ymax, ymax)).
__global__ __launch_bounds__(256) void k_mlp_infer(const MlpPacked* __restrict__ W, const float* __restrict__ X,
                                                   int64_t n, float* __restrict__ y, double* __restrict__ H,
                                                   float ymax)
{
    __shared__ float sb[4][NH];
    __shared__ float sx[2][NIN];
    for (int t = threadIdx.x; t < NH; t += blockDim.x) {
        sb[0][t] = W->b1[t];
        sb[1][t] = W->b2[t];
        sb[2][t] = W->b3[t];
        sb[3][t] = W->w4[t];
    }
    for (int t = threadIdx.x; t < NIN; t += blockDim.x) {
        sx[0][t] = W->xmu[t];
        sx[1][t] = W->rxsd[t];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    bf16x4 a1[4], a2[4][4], a3[4][4];
    for (int t = 0; t < 4; t++) {
        a1[t] = W->a1[t][lane];
        for (int k = 0; k < 4; k++) {
            a2[t][k] = W->a2[t][k][lane];
            a3[t][k] = W->a3[t][k][lane];
        }
    }
    const float b4 = W->b4, ymu = W->ymu, ysd = W->ysd;
    const int64_t n_tiles = (n + 15) / 16;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
        const int64_t p = tile * 16 + col;
        const bool ok = p < n;
        // inputs 4g..4g+3 of particle p (inputs from SPH_MLP_XSTRIDE on are zero)
        float v[4];
        if (g < 2) {
            float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ok) q = *(const float4*)(X + p * XS + 4 * g);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
            v[0] = v[1] = v[2] = v[3] = 0.f;
        }
        for (int j = 0; j < 4; j++) v[j] = (v[j] - sx[0][4 * g + j]) * sx[1][4 * g + j];
        bf16x4 bh[4], bl[4];
        split4(v, bh[0], bl[0]);
        f32x4 acc[4];
        for (int t = 0; t < 4; t++) {
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[t] = MFMA16(a1[t], bh[0], acc[t]);
            acc[t] = MFMA16(a1[t], bl[0], acc[t]);
        }
        for (int t = 0; t < 4; t++) {
            float h[4];
            for (int j = 0; j < 4; j++) h[j] = silu_f(acc[t][j] + sb[0][16 * t + 4 * g + j]);
            split4(h, bh[t], bl[t]);
        }
        for (int t = 0; t < 4; t++) {
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int k = 0; k < 4; k++) {
                acc[t] = MFMA16(a2[t][k], bh[k], acc[t]);
                acc[t] = MFMA16(a2[t][k], bl[k], acc[t]);
            }
        }
        for (int t = 0; t < 4; t++) {
            float h[4];
            for (int j = 0; j < 4; j++) h[j] = silu_f(acc[t][j] + sb[1][16 * t + 4 * g + j]);
            split4(h, bh[t], bl[t]);
        }
        for (int t = 0; t < 4; t++) {
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int k = 0; k < 4; k++) {
                acc[t] = MFMA16(a3[t][k], bh[k], acc[t]);
                acc[t] = MFMA16(a3[t][k], bl[k], acc[t]);
            }
        }
        float part = 0.f;
        for (int t = 0; t < 4; t++)
            for (int j = 0; j < 4; j++) part += silu_f(acc[t][j] + sb[2][16 * t + 4 * g + j]) * sb[3][16 * t + 4 * g + j];
        // the four lane groups hold the four quarters of the hidden units
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0 && ok) {
            const float yv = ymu + ysd * (part + b4);
            if (y) y[p] = yv;
            if (H) {
                const float yc = fminf(fmaxf(yv, -ymax), ymax);
                const double hp = H[p];
                H[p] = isfinite(yc) ? hp * exp((double)yc) : hp;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Training: float32 forward and backward over micro-batches of MB rows per
// workgroup (weights rounded to bfloat16 as in inference), partial
// gradients per workgroup, then a reduction fused with Adam.
// ---------------------------------------------------------------------------
#define MB 32
// Workgroups of k_mlp_fb at most: one per compute unit (about 88 KB of LDS
// each); each loops over row tiles of MB rows.
#define MLP_FB_WGS 256

struct TrainArgs {
    const float* p;          // parameter vector (float32 masters)
    const float* X;          // rows, stride SPH_MLP_XSTRIDE
    const float* y;          // targets
    int64_t N;               // rows in the data set
    int64_t row0;            // first position of this minibatch in the permuted order
    int64_t count;           // rows in this minibatch
    uint64_t pa, pb;         // row = (pa * pos + pb) mod N
    float inv_count;         // 1 / rows of the minibatch
    float* part;             // [workgroups][NT] partial gradients
    float* part_loss;        // [workgroups]
};

// Workgroups of one k_mlp_fb launch over `count` rows.
inline int fb_workgroups(int64_t count)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((count + MB - 1) / MB, MLP_FB_WGS));
}

__global__ __launch_bounds__(256) void k_mlp_fb(TrainArgs a)
{
    __shared__ float W1[NIN * NH], W2[NH * NH], W3[NH * NH];
    __shared__ float bb[3][NH], w4[NH], xmu[NIN], rxsd[NIN];
    __shared__ float xh[MB][NIN];
    __shared__ float hA[3][MB][NH];   // activations h1, h2, h3
    __shared__ float dA[3][MB][NH];   // SiLU'(z), then dL/dz
    __shared__ float dout[MB], red[MB];
    const int tid = threadIdx.x;
    for (int i = tid; i < NIN * NH; i += 256) W1[i] = bf16r(a.p[O_W1 + i]);
    for (int i = tid; i < NH * NH; i += 256) {
        W2[i] = bf16r(a.p[O_W2 + i]);
        W3[i] = bf16r(a.p[O_W3 + i]);
    }
    if (tid < NH) {
        bb[0][tid] = a.p[O_B1 + tid];
        bb[1][tid] = a.p[O_B2 + tid];
        bb[2][tid] = a.p[O_B3 + tid];
        w4[tid] = bf16r(a.p[O_W4 + tid]);
    }
    if (tid < NIN) {
        xmu[tid] = a.p[O_XMU + tid];
        rxsd[tid] = 1.0f / a.p[O_XSD + tid];
    }
    const float b4 = a.p[O_B4], ymu = a.p[O_YMU], rysd = 1.0f / a.p[O_YSD];
    const int s = tid >> 3, q = tid & 7;   // sample, eighth of the units
    // this thread's share of the gradient, summed over the workgroup's tiles:
    // W2, W3 row kw = tid/4, columns 16 (tid%4) .. +15; W1 row k1 = tid/16,
    // columns 4 (tid%16) .. +3; unit tid of b1, b2, b3, w4 (tid < NH); b4
    // and the loss (tid 0)
    const int kw = tid >> 2, c0 = 16 * (tid & 3);
    const int k1 = tid >> 4, c1 = 4 * (tid & 15);
    float accW[2][16], acc1[4] = {0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 16; j++) accW[0][j] = accW[1][j] = 0.f;
    float g1 = 0.f, g2 = 0.f, g3 = 0.f, g4 = 0.f, gb = 0.f, Lsum = 0.f;
    const int64_t n_tiles = (a.count + MB - 1) / MB;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t pos = tile * MB + s;
        const bool valid = pos < a.count;
        int64_t row = 0;
        if (valid) {
            // N < 2^31, so the product stays below 2^62
            const uint64_t k = (uint64_t)(a.row0 + pos) % (uint64_t)a.N;
            row = (int64_t)((a.pa * k + a.pb) % (uint64_t)a.N);
        }
        // weights loaded; the previous tile's readers of xh, hA, dA are done
        __syncthreads();
        // standardised inputs: thread (s, q) loads inputs 2q, 2q+1
        for (int j = 0; j < 2; j++) {
            const int k = 2 * q + j;
            const float raw = (valid && k < XS) ? a.X[row * XS + k] : 0.f;
            xh[s][k] = valid ? (raw - xmu[k]) * rxsd[k] : 0.f;
        }
        __syncthreads();
        // forward: thread (s, q) computes units 8q..8q+7 of sample s
        for (int l = 0; l < 3; l++) {
            float z[8];
            for (int j = 0; j < 8; j++) z[j] = bb[l][8 * q + j];
            if (l == 0) {
                for (int k = 0; k < NIN; k++) {
                    const float x = xh[s][k];
                    for (int j = 0; j < 8; j++) z[j] += x * W1[k * NH + 8 * q + j];
                }
            } else {
                const float* Wl = l == 1 ? W2 : W3;
                for (int k = 0; k < NH; k++) {
                    const float x = hA[l - 1][s][k];
                    for (int j = 0; j < 8; j++) z[j] += x * Wl[k * NH + 8 * q + j];
                }
            }
            for (int j = 0; j < 8; j++) {
                hA[l][s][8 * q + j] = silu_f(z[j]);
                dA[l][s][8 * q + j] = dsilu_f(z[j]);
            }
            __syncthreads();
        }
        // output and dL/do
        float part = 0.f;
        for (int j = 0; j < 8; j++) part += hA[2][s][8 * q + j] * w4[8 * q + j];
        part += __shfl_xor(part, 1);
        part += __shfl_xor(part, 2);
        part += __shfl_xor(part, 4);
        if (q == 0) {
            float r = 0.f;
            if (valid) r = part + b4 - (a.y[row] - ymu) * rysd;
            dout[s] = r * a.inv_count;
            red[s] = 0.5f * r * r;
        }
        __syncthreads();
        // backward through the layers: dA[l] becomes dL/dz_l
        for (int j = 0; j < 8; j++) dA[2][s][8 * q + j] *= dout[s] * w4[8 * q + j];
        __syncthreads();
        for (int l = 2; l >= 1; l--) {
            const float* Wl = l == 2 ? W3 : W2;
            float dh[8];
            for (int j = 0; j < 8; j++) dh[j] = 0.f;
            for (int k = 0; k < NH; k++) {
                const float d = dA[l][s][k];
                for (int j = 0; j < 8; j++) dh[j] += d * Wl[(8 * q + j) * NH + k];
            }
            for (int j = 0; j < 8; j++) dA[l - 1][s][8 * q + j] *= dh[j];
            __syncthreads();
        }
        // this tile's contribution to the gradient
        for (int l = 1; l <= 2; l++)
            for (int r = 0; r < MB; r++) {
                const float hv = hA[l - 1][r][kw];
                for (int j = 0; j < 16; j++) accW[l - 1][j] += hv * dA[l][r][c0 + j];
            }
        for (int r = 0; r < MB; r++) {
            const float xv = xh[r][k1];
            for (int j = 0; j < 4; j++) acc1[j] += xv * dA[0][r][c1 + j];
        }
        if (tid < NH)
            for (int r = 0; r < MB; r++) {
                g1 += dA[0][r][tid];
                g2 += dA[1][r][tid];
                g3 += dA[2][r][tid];
                g4 += hA[2][r][tid] * dout[r];
            }
        if (tid == 0)
            for (int r = 0; r < MB; r++) {
                gb += dout[r];
                Lsum += red[r];
            }
    }
    // partial gradients of this workgroup (every one of the NT entries)
    float* G = a.part + (size_t)blockIdx.x * NT;
    for (int j = 0; j < 16; j++) {
        G[O_W2 + kw * NH + c0 + j] = accW[0][j];
        G[O_W3 + kw * NH + c0 + j] = accW[1][j];
    }
    for (int j = 0; j < 4; j++) G[O_W1 + k1 * NH + c1 + j] = acc1[j];
    if (tid < NH) {
        G[O_B1 + tid] = g1;
        G[O_B2 + tid] = g2;
        G[O_B3 + tid] = g3;
        G[O_W4 + tid] = g4;
    }
    if (tid == 0) {
        G[O_B4] = gb;
        a.part_loss[blockIdx.x] = Lsum;
    }
}

// Sum of the workgroup partials; then either store the gradient or apply
// one Adam step (adam != 0).  Thread 0 also sums the loss.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, const float* __restrict__ part_loss,
                                                    int nwg, float inv_count, float* grad, float* p, float* m, float* v,
                                                    int adam, float lr, float b1, float b2, float eps, float c1,
                                                    float c2, float* loss_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NT) {
        float g = 0.f;
        for (int w = 0; w < nwg; w++) g += part[(size_t)w * NT + i];
        if (grad) grad[i] = g;
        if (adam) {
            const float mi = b1 * m[i] + (1.f - b1) * g;
            const float vi = b2 * v[i] + (1.f - b2) * g * g;
            m[i] = mi;
            v[i] = vi;
            p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        }
    }
    if (i == 0 && loss_out) {
        double L = 0.0;
        for (int w = 0; w < nwg; w++) L += part_loss[w];
        *loss_out = (float)(L * inv_count);
    }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* p, float* m, float* v, const float* __restrict__ g, float lr,
                                                  float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NT) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------
__device__ inline void feat_cell(const FeatGrid& F, double x, double y, double z, int c[3], double f[3])
{
    const double p[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        const double u = p[a] * F.scale[a];
        int k = (int)floor(u);
        k = k < 0 ? 0 : (k > F.G[a] - 1 ? F.G[a] - 1 : k);
        c[a] = k;
        f[a] = u - k;
    }
}

__global__ __launch_bounds__(256) void k_feat_hist(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                                   const double* __restrict__ z, const int32_t* __restrict__ dom,
                                                   const FeatGrid* __restrict__ fg, int* cnt)
{
    // particles arrive in the Morton order of the last cell build, so runs of
    // lanes share a cell: one atomic per run
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    long long cell = -1 - lane;  // distinct for inactive lanes
    if (i < n) {
        const FeatGrid& F = fg[dom ? dom[i] : 0];
        int c[3];
        double f[3];
        feat_cell(F, x[i], y[i], z[i], c, f);
        cell = F.off + ((long long)c[0] * F.G[1] + c[1]) * F.G[2] + c[2];
    }
    const long long prev = __shfl_up(cell, 1);
    const bool head = lane == 0 || prev != cell;
    const uint64_t heads = __ballot(head);
    if (i < n && head) {
        // run length: distance to the next head (or the wave end)
        const uint64_t above = lane == 63 ? 0ull : heads >> (lane + 1);
        const int len = above ? __ffsll((long long)above) : 64 - lane;
        atomicAdd(&cnt[cell], len);
    }
}

__global__ __launch_bounds__(256) void k_features(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                                  const double* __restrict__ z, const double* __restrict__ vx,
                                                  const double* __restrict__ vy, const double* __restrict__ vz,
                                                  const double* __restrict__ H, const double* __restrict__ rho,
                                                  const double* __restrict__ P, const double* __restrict__ dudt,
                                                  const int32_t* __restrict__ dom, const FeatGrid* __restrict__ fg,
                                                  const int* __restrict__ cnt, double dt, float* __restrict__ X,
                                                  double* __restrict__ hprev)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FeatGrid& F = fg[dom ? dom[i] : 0];
    int c[3];
    double fr[3];
    feat_cell(F, x[i], y[i], z[i], c, fr);
    long long s27 = 0, sp[3] = {0, 0, 0}, sm[3] = {0, 0, 0};
    for (int dx = -1; dx <= 1; dx++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dz = -1; dz <= 1; dz++) {
                const int d[3] = {dx, dy, dz};
                int e[3];
                for (int a = 0; a < 3; a++) {
                    e[a] = (c[a] + d[a]) % F.G[a];
                    if (e[a] < 0) e[a] += F.G[a];
                }
                const int v = cnt[F.off + ((int64_t)e[0] * F.G[1] + e[1]) * F.G[2] + e[2]];
                s27 += v;
                for (int a = 0; a < 3; a++) {
                    if (d[a] == 1) sp[a] += v;
                    else if (d[a] == -1) sm[a] += v;
                }
            }
    const int own = cnt[F.off + ((int64_t)c[0] * F.G[1] + c[1]) * F.G[2] + c[2]];
    const double h = H[i];
    double g[3], g2 = 0.0, gf = 0.0;
    for (int a = 0; a < 3; a++) {
        g[a] = (double)(sp[a] - sm[a]) / (double)s27;
        g2 += g[a] * g[a];
        gf += g[a] * (fr[a] - 0.5);
    }
    const double Pi = P[i];
    const double comp = Pi > 0.0 ? -dt * rho[i] * dudt[i] / (3.0 * Pi) : 0.0;
    const double vv = sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    float* row = X + i * XS;
    row[0] = (float)log(h / F.sbox);
    row[1] = (float)log((double)own);
    row[2] = (float)log((double)s27 / (27.0 * F.nbar));
    row[3] = (float)sqrt(g2);
    row[4] = (float)gf;
    row[5] = (float)comp;
    row[6] = (float)(dt * vv / h);
    row[7] = 0.f;
    if (hprev) hprev[i] = h;
}

// Moments of the recorded samples (inputs and target) for standardisation.
__global__ __launch_bounds__(256) void k_moments(int64_t n, const float* __restrict__ X, const float* __restrict__ y,
                                                 double* __restrict__ out)
{
    __shared__ double s[2 * (XS + 1)][4];
    double acc[2 * (XS + 1)];
    for (int k = 0; k < 2 * (XS + 1); k++) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < XS; k++) {
            const double v = X[i * XS + k];
            acc[2 * k] += v;
            acc[2 * k + 1] += v * v;
        }
        const double v = y[i];
        acc[2 * XS] += v;
        acc[2 * XS + 1] += v * v;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < 2 * (XS + 1); k++) {
        double v = acc[k];
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) s[k][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2 * (XS + 1)) {
        const double v = s[threadIdx.x][0] + s[threadIdx.x][1] + s[threadIdx.x][2] + s[threadIdx.x][3];
        atomicAdd(&out[threadIdx.x], v);
    }
}

// Sample recording: particle i of step `step` is kept when a hash of (seed,
// step, id) falls below rate; slots are taken with one atomic per wave.
__device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_record(int64_t n, const float* __restrict__ X, const double* __restrict__ H,
                                                const double* __restrict__ hprev, const int64_t* __restrict__ id,
                                                uint64_t seed, uint64_t step, double rate, float* dsX, float* dsy,
                                                unsigned int cap, unsigned int* counter)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool sel = false;
    if (i < n) {
        const uint64_t key = id ? (uint64_t)id[i] : (uint64_t)i;
        const uint64_t h = mix64(seed ^ mix64(step ^ mix64(key)));
        sel = (double)(h >> 11) * (1.0 / 9007199254740992.0) < rate;
    }
    const uint64_t mask = __ballot(sel);
    const int cnt = __popcll(mask);
    unsigned int base = 0;
    if (lane == 0 && cnt) base = atomicAdd(counter, (unsigned int)cnt);
    base = __shfl(base, 0);
    const int below = __popcll(mask & ((1ull << lane) - 1ull));
    const unsigned int slot = base + below;
    if (sel && slot < cap) {
        for (int k = 0; k < XS; k++) dsX[(size_t)slot * XS + k] = X[i * XS + k];
        dsy[slot] = (float)log(H[i] / hprev[i]);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static sph_status pack(const float* p, MlpPacked* w, hipStream_t s)
{
    k_mlp_pack<<<nblocks(4 * 64 + 2 * 16 * 64, 256), 256, 0, s>>>(p, w);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

static int infer_grid(int64_t n)
{
    const int64_t tiles = (n + 15) / 16;
    return (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 256 * 8));
}

// gradient (and optional Adam step) of one minibatch
struct TrainScratch {
    DevBuf part, part_loss, loss;
};

// Forward + backward over `count` rows into nwg = fb_workgroups(count)
// workgroup partials (part: nwg x NT floats, part_loss: nwg floats), then
// their sum into grad and/or one Adam step.
static sph_status fb_reduce(float* part, float* part_loss, const float* p, const float* X, const float* y, int64_t N,
                            int64_t row0, int64_t count, uint64_t pa, uint64_t pb, float* grad, float* pw, float* m,
                            float* v, bool adam, float lr, float b1, float b2, float eps, int t, float* loss_slot,
                            hipStream_t s)
{
    const int nwg = fb_workgroups(count);
    TrainArgs a;
    a.p = p;
    a.X = X;
    a.y = y;
    a.N = N;
    a.row0 = row0;
    a.count = count;
    a.pa = pa;
    a.pb = pb;
    a.inv_count = 1.0f / (float)count;
    a.part = part;
    a.part_loss = part_loss;
    k_mlp_fb<<<nwg, 256, 0, s>>>(a);
    SPH_CHECK_LAUNCH();
    const float c1 = adam ? (float)(1.0 - pow((double)b1, t)) : 1.f;
    const float c2 = adam ? (float)(1.0 - pow((double)b2, t)) : 1.f;
    k_mlp_reduce<<<nblocks(NT, 256), 256, 0, s>>>(part, part_loss, nwg, 1.0f / (float)count, grad, pw, m, v,
                                                   adam ? 1 : 0, lr, b1, b2, eps, c1, c2, loss_slot);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

static sph_status minibatch(TrainScratch& S, const float* p, const float* X, const float* y, int64_t N, int64_t row0,
                            int64_t count, uint64_t pa, uint64_t pb, float* grad, float* pw, float* m, float* v,
                            bool adam, float lr, float b1, float b2, float eps, int t, float* loss_slot, hipStream_t s)
{
    const int nwg = fb_workgroups(count);
    SPH_TRY(buf_ensure(S.part, (size_t)nwg * NT * sizeof(float)));
    SPH_TRY(buf_ensure(S.part_loss, (size_t)nwg * sizeof(float)));
    return fb_reduce((float*)S.part.p, (float*)S.part_loss.p, p, X, y, N, row0, count, pa, pb, grad, pw, m, v, adam,
                     lr, b1, b2, eps, t, loss_slot, s);
}

static uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

static uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Feature grids of the boxes (counts per box from the last cell build).
static sph_status feat_setup(sph_ctx* c)
{
    const int nd = c->prm.n_domains;
    if (c->fgrid_h.size() == (size_t)nd && c->fgrid_n == c->n) return SPH_OK;
    std::vector<int> rng(nd + 1);
    SPH_CHECK_HIP(hipMemcpyAsync(rng.data(), c->dranges.p, (nd + 1) * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    c->fgrid_h.assign(nd, FeatGrid{});
    int64_t off = 0;
    for (int d = 0; d < nd; d++) {
        FeatGrid& F = c->fgrid_h[d];
        const double* L = &c->boxes[3 * d];
        const int64_t nb = std::max(rng[d + 1] - rng[d], 0);
        const double vol = L[0] * L[1] * L[2];
        const double s = 2.0 * pow(vol / (double)std::max<int64_t>(nb, 1), 1.0 / 3.0);
        int64_t cells = 1;
        for (int a = 0; a < 3; a++) {
            F.G[a] = (int)std::min(256.0, std::max(1.0, floor(L[a] / s + 0.5)));
            F.scale[a] = (double)F.G[a] / L[a];
            cells *= F.G[a];
        }
        F.sbox = pow(vol / (double)std::max<int64_t>(nb, 1), 1.0 / 3.0);
        F.nbar = (double)nb / (double)cells;
        F.off = off;
        off += cells;
    }
    c->fgrid_cells = off;
    c->fgrid_n = c->n;
    SPH_TRY(buf_ensure(c->fgrid, nd * sizeof(FeatGrid)));
    SPH_TRY(buf_ensure(c->fcount, (size_t)off * sizeof(int)));
    SPH_CHECK_HIP(hipMemcpyAsync(c->fgrid.p, c->fgrid_h.data(), nd * sizeof(FeatGrid), hipMemcpyHostToDevice,
                                 c->stream));
    return SPH_OK;
}

sph_status mlp_features(sph_ctx* c, double dt, float* X, double* hprev)
{
    SPH_TRY(feat_setup(c));
    SPH_CHECK_HIP(hipMemsetAsync(c->fcount.p, 0, (size_t)c->fgrid_cells * sizeof(int), c->stream));
    const int nb = nblocks(c->n, 256);
    k_feat_hist<<<nb, 256, 0, c->stream>>>(c->n, c->P.x, c->P.y, c->P.z, c->P.domain, (const FeatGrid*)c->fgrid.p,
                                          (int*)c->fcount.p);
    SPH_CHECK_LAUNCH();
    k_features<<<nb, 256, 0, c->stream>>>(c->n, c->P.x, c->P.y, c->P.z, c->P.vx, c->P.vy, c->P.vz, c->P.H, c->P.rho,
                                         c->P.P, c->P.dudt, c->P.domain, (const FeatGrid*)c->fgrid.p,
                                         (const int*)c->fcount.p, dt, X, hprev);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

// Step hook before the cell rebuild: features of the drifted particles,
// previous H saved, and (predictor on) H replaced by the prediction.
sph_status mlp_pre_build(sph_ctx* c, double dt)
{
    c->mlp_pending = false;
    c->pev_done = false;
    const bool use = c->h_pred && c->mlp_ready;
    if (!use && !c->rec_on) return SPH_OK;
    if (!c->pev[0]) {
        SPH_CHECK_HIP(hipEventCreate(&c->pev[0]));
        SPH_CHECK_HIP(hipEventCreate(&c->pev[1]));
    }
    SPH_CHECK_HIP(hipEventRecord(c->pev[0], c->stream));
    SPH_TRY(buf_ensure(c->mlp_X, (size_t)c->n * XS * sizeof(float)));
    if (c->rec_on) SPH_TRY(buf_ensure(c->mlp_hprev, (size_t)c->n * sizeof(double)));
    SPH_TRY(mlp_features(c, dt, (float*)c->mlp_X.p, c->rec_on ? (double*)c->mlp_hprev.p : nullptr));
    if (use) {
        k_mlp_infer<<<infer_grid(c->n), 256, 0, c->stream>>>((const MlpPacked*)c->mlp_packed.p,
                                                             (const float*)c->mlp_X.p, c->n, nullptr, c->P.H, 0.25f);
        SPH_CHECK_LAUNCH();
    }
    SPH_CHECK_HIP(hipEventRecord(c->pev[1], c->stream));
    c->pev_done = true;
    // features and previous H follow the particles through the rebuild only
    // when they are recorded after the density stage
    c->mlp_pending = c->rec_on;
    return SPH_OK;
}

// Step hook after the force stage: record samples of converged H.
sph_status mlp_post_step(sph_ctx* c)
{
    if (c->mlp_pending && c->rec_on && c->rec_cap > 0) {
        k_record<<<nblocks(c->n, 256), 256, 0, c->stream>>>(
            c->n, (const float*)c->mlp_X.p, c->P.H, (const double*)c->mlp_hprev.p, c->P.id, c->rec_seed,
            (uint64_t)c->step_count, c->rec_rate, c->ds_X, c->ds_y, (unsigned int)c->rec_cap,
            (unsigned int*)c->ds_count.p);
        SPH_CHECK_LAUNCH();
    }
    c->mlp_pending = false;
    return SPH_OK;
}

static sph_status ensure_params(sph_ctx* c)
{
    SPH_TRY(buf_ensure(c->mlp_params, NP * sizeof(float)));
    SPH_TRY(buf_ensure(c->mlp_packed, sizeof(MlpPacked)));
    SPH_TRY(buf_ensure(c->mlp_m, NT * sizeof(float)));
    SPH_TRY(buf_ensure(c->mlp_v, NT * sizeof(float)));
    return SPH_OK;
}

extern "C" {

// Scratch of the context-free calls over n rows: packed weights, partial
// gradients of each workgroup (k_mlp_fb, MB rows each) and the loss slot.
static size_t mlp_scratch_bytes(int64_t n)
{
    const size_t nwg = (size_t)fb_workgroups(n);
    const size_t r = 256;
    auto up = [&](size_t b) { return (b + r - 1) / r * r + r; };
    return up(sizeof(MlpPacked)) + up(nwg * NT * sizeof(float)) + up(nwg * sizeof(float)) + up(sizeof(float)) +
           ((size_t)4 << 10);
}

sph_status sph_mlp_workspace_size(int64_t n, size_t* bytes)
{
    if (n < 0 || !bytes) return SPH_ERR_INVALID;
    *bytes = mlp_scratch_bytes(n);
    return SPH_OK;
}

sph_status sph_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* workspace, size_t bytes,
                           void* hip_stream)
{
    if (n < 0 || ((!params || !X || !y) && n > 0)) return SPH_ERR_INVALID;
    if (n == 0) return SPH_OK;
    if (!workspace) return SPH_ERR_INVALID;
    const hipStream_t s = (hipStream_t)hip_stream;
    Pool pool;
    pool.init(workspace, bytes);
    PoolScope ps(&pool);
    DevBuf w;
    SPH_TRY(buf_ensure(w, sizeof(MlpPacked)));
    SPH_TRY(pack(params, (MlpPacked*)w.p, s));
    k_mlp_infer<<<infer_grid(n), 256, 0, s>>>((const MlpPacked*)w.p, X, n, y, nullptr, 0.f);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

sph_status sph_mlp_loss_grad(const float* params, const float* X, const float* y, int64_t n, float* grad,
                             double* loss, void* workspace, size_t bytes, void* hip_stream)
{
    if (n <= 0 || n > SPH_MLP_MAX_ROWS || !params || !X || !y || !grad || !workspace) return SPH_ERR_INVALID;
    const hipStream_t s = (hipStream_t)hip_stream;
    Pool pool;
    pool.init(workspace, bytes);
    PoolScope ps(&pool);
    TrainScratch S;
    SPH_TRY(buf_ensure(S.loss, sizeof(float)));
    SPH_TRY(minibatch(S, params, X, y, n, 0, n, 1, 0, grad, nullptr, nullptr, nullptr, false, 0.f, 0.f, 0.f, 0.f, 0,
                      (float*)S.loss.p, s));
    float L = 0.f;
    SPH_CHECK_HIP(hipMemcpyAsync(&L, S.loss.p, sizeof(float), hipMemcpyDeviceToHost, s));
    SPH_CHECK_HIP(hipStreamSynchronize(s));
    if (loss) *loss = L;
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// sph_mlp_loss_grad without a workspace.  The workgroup partials and the loss
// live in `scratch`, a fixed array of this library that every GPU holds
// once (MLP_FB_WGS x NT partial gradients, MLP_FB_WGS partial losses, the
// loss): about 9.7 MB, enough for any row count since k_mlp_fb runs at most
// MLP_FB_WGS workgroups.  Every call on one GPU shares that GPU's copy.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_PART = (size_t)MLP_FB_WGS * NT;
constexpr size_t NOALLOC_FLOATS = NOALLOC_PART + MLP_FB_WGS + 64;
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of the current device's copy of `scratch` (its host-side
// name is not a device address), looked up on the first call on a device.
static sph_status scratch_address(float** out)
{
    int dev = -1;
    SPH_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SPH_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        SPH_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return SPH_ERR_HIP;
        g_scratch_ptr[dev] = (float*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return SPH_OK;
}

sph_status sph_mlp_loss_grad_noalloc(const float* params, const float* X, const float* y, int64_t n, float* grad,
                                     double* loss, void* hip_stream)
{
    if (n <= 0 || n > SPH_MLP_MAX_ROWS || !params || !X || !y || !grad) return SPH_ERR_INVALID;
    static_assert((size_t)MLP_FB_WGS * NT + MLP_FB_WGS + 1 <= NOALLOC_FLOATS, "scratch too small");
    if ((size_t)fb_workgroups(n) > MLP_FB_WGS) return SPH_ERR_WORKSPACE;
    float* ptr = nullptr;
    SPH_TRY(scratch_address(&ptr));
    const hipStream_t s = (hipStream_t)hip_stream;
    // every partial and the loss are written before they are read: nothing
    // in the array needs clearing between calls
    float* part = ptr;
    float* part_loss = ptr + NOALLOC_PART;
    float* loss_slot = part_loss + MLP_FB_WGS;
    SPH_TRY(fb_reduce(part, part_loss, params, X, y, n, 0, n, 1, 0, grad, nullptr, nullptr, nullptr, false, 0.f, 0.f,
                      0.f, 0.f, 0, loss_slot, s));
    float L = 0.f;
    SPH_CHECK_HIP(hipMemcpyAsync(&L, loss_slot, sizeof(float), hipMemcpyDeviceToHost, s));
    SPH_CHECK_HIP(hipStreamSynchronize(s));
    if (loss) *loss = L;
    return SPH_OK;
}

sph_status sph_mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr, float beta1,
                        float beta2, float eps, void* hip_stream)
{
    if (!params || !m || !v || !grad || t < 1) return SPH_ERR_INVALID;
    const float c1 = (float)(1.0 - pow((double)beta1, t)), c2 = (float)(1.0 - pow((double)beta2, t));
    k_mlp_adam<<<nblocks(NT, 256), 256, 0, (hipStream_t)hip_stream>>>(params, m, v, grad, lr, beta1, beta2, eps, c1,
                                                                       c2);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

sph_status sph_h_features(sph_ctx* c, double dt, float* X)
{
    if (!c || !X) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->built) return SPH_ERR_STATE;
    return mlp_features(c, dt, X, nullptr);
}

sph_status sph_h_record(sph_ctx* c, float* X, float* y, int64_t capacity, double rate, uint64_t seed,
                        int64_t* held)
{
    if (!c || capacity < 0 || capacity > INT32_MAX || !(rate >= 0.0 && rate <= 1.0)) return SPH_ERR_INVALID;
    if (capacity > 0 && (!X || !y)) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (capacity == 0) {
        c->rec_on = false;
        c->rec_cap = 0;
        c->ds_X = nullptr;
        c->ds_y = nullptr;
        if (held) *held = 0;
        return SPH_OK;
    }
    if (!c->rec_on || capacity != c->rec_cap || X != c->ds_X || y != c->ds_y) {
        SPH_TRY(buf_ensure(c->ds_count, sizeof(unsigned int)));
        SPH_CHECK_HIP(hipMemsetAsync(c->ds_count.p, 0, sizeof(unsigned int), c->stream));
    }
    c->ds_X = X;
    c->ds_y = y;
    c->rec_on = true;
    c->rec_cap = capacity;
    c->rec_rate = rate;
    c->rec_seed = seed;
    if (held) {
        unsigned int h = 0;
        SPH_CHECK_HIP(hipMemcpyAsync(&h, c->ds_count.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
        *held = std::min<int64_t>(h, capacity);
    }
    return SPH_OK;
}

sph_status sph_h_train(sph_ctx* c, int epochs, int batch, double lr, uint64_t seed, int init, double* loss)
{
    if (!c || epochs < 0 || batch < 1 || !(lr > 0.0)) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    if (!c->ds_count.p || c->rec_cap <= 0) return SPH_ERR_STATE;
    unsigned int h = 0;
    SPH_CHECK_HIP(hipMemcpyAsync(&h, c->ds_count.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    const int64_t N = std::min<int64_t>(h, c->rec_cap);
    if (N < 2) return SPH_ERR_STATE;
    if (!init && !c->mlp_have) return SPH_ERR_STATE;
    SPH_TRY(ensure_params(c));
    const float* dX = c->ds_X;
    const float* dy = c->ds_y;
    if (init) {
        // standardisation from the samples, fresh weights, zero moments
        DevBuf mom;
        SPH_TRY(buf_ensure(mom, 2 * (XS + 1) * sizeof(double)));
        SPH_CHECK_HIP(hipMemsetAsync(mom.p, 0, 2 * (XS + 1) * sizeof(double), c->stream));
        k_moments<<<std::min(nblocks(N, 256), 1024), 256, 0, c->stream>>>(N, dX, dy, (double*)mom.p);
        SPH_CHECK_LAUNCH();
        double mh[2 * (XS + 1)];
        SPH_CHECK_HIP(hipMemcpyAsync(mh, mom.p, sizeof(mh), hipMemcpyDeviceToHost, c->stream));
        SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
        buf_free(mom);
        std::vector<float> p(NP, 0.f);
        uint64_t st = seed;
        auto uni = [&](double a) { return (float)(a * (2.0 * ((double)(splitmix(st) >> 11) / 9007199254740992.0) - 1.0)); };
        for (int i = 0; i < NIN * NH; i++) p[O_W1 + i] = uni(sqrt(3.0 / NIN));
        for (int i = 0; i < NH * NH; i++) p[O_W2 + i] = uni(sqrt(3.0 / NH));
        for (int i = 0; i < NH * NH; i++) p[O_W3 + i] = uni(sqrt(3.0 / NH));
        for (int i = 0; i < NH; i++) p[O_W4 + i] = uni(sqrt(3.0 / NH));
        for (int k = 0; k < NIN; k++) {
            double mu = 0.0, sd = 1.0;
            if (k < XS) {
                mu = mh[2 * k] / N;
                const double var = mh[2 * k + 1] / N - mu * mu;
                sd = var > 1e-24 * (1.0 + mu * mu) ? sqrt(var) : 1.0;
            }
            p[O_XMU + k] = (float)mu;
            p[O_XSD + k] = (float)sd;
        }
        {
            const double mu = mh[2 * XS] / N;
            const double var = mh[2 * XS + 1] / N - mu * mu;
            p[O_YMU] = (float)mu;
            p[O_YSD] = (float)(var > 1e-30 ? sqrt(var) : 1.0);
        }
        SPH_CHECK_HIP(hipMemcpyAsync(c->mlp_params.p, p.data(), NP * sizeof(float), hipMemcpyHostToDevice, c->stream));
        SPH_CHECK_HIP(hipMemsetAsync(c->mlp_m.p, 0, NT * sizeof(float), c->stream));
        SPH_CHECK_HIP(hipMemsetAsync(c->mlp_v.p, 0, NT * sizeof(float), c->stream));
        c->adam_t = 0;
        c->mlp_have = true;
    }
    const int64_t B = std::min<int64_t>(batch, N);
    const int64_t steps_per_epoch = (N + B - 1) / B;
    TrainScratch S;
    SPH_TRY(buf_ensure(S.loss, (size_t)std::max<int64_t>(steps_per_epoch, 1) * sizeof(float)));
    uint64_t rs = seed ^ 0xD1B54A32D192ED03ull;
    float* p = (float*)c->mlp_params.p;
    sph_status st = SPH_OK;
    for (int e = 0; e < epochs && st == SPH_OK; e++) {
        // affine permutation of the sample order for this epoch
        uint64_t pa = 1 + splitmix(rs) % (uint64_t)N;
        while (gcd_u64(pa, (uint64_t)N) != 1) pa = 1 + (pa % (uint64_t)N);
        const uint64_t pb = splitmix(rs) % (uint64_t)N;
        for (int64_t k = 0; k < steps_per_epoch && st == SPH_OK; k++) {
            const int64_t row0 = k * B;
            const int64_t cnt = std::min<int64_t>(B, N - row0);
            c->adam_t++;
            st = minibatch(S, p, dX, dy, N, row0, cnt, pa, pb, nullptr, p, (float*)c->mlp_m.p, (float*)c->mlp_v.p,
                           true, (float)lr, 0.9f, 0.999f, 1e-8f, c->adam_t, (float*)S.loss.p + k, c->stream);
        }
    }
    if (st == SPH_OK && loss) {
        std::vector<float> L((size_t)steps_per_epoch);
        if (hipMemcpyAsync(L.data(), S.loss.p, L.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess)
            st = SPH_ERR_HIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess) st = SPH_ERR_HIP;
        double sL = 0.0;
        for (float v : L) sL += v;
        *loss = epochs > 0 ? sL / (double)L.size() : 0.0;
    }
    buf_free(S.part);
    buf_free(S.part_loss);
    buf_free(S.loss);
    if (st == SPH_OK) st = pack(p, (MlpPacked*)c->mlp_packed.p, c->stream);
    if (st == SPH_OK) c->mlp_ready = true;
    return st;
}

sph_status sph_h_set_params(sph_ctx* c, const float* params)
{
    if (!c || !params) return SPH_ERR_INVALID;
    PoolScope ps(&c->pool);
    for (int k = 0; k < NIN; k++)
        if (!(params[O_XSD + k] != 0.0f)) return SPH_ERR_INVALID;
    if (!(params[O_YSD] == params[O_YSD])) return SPH_ERR_INVALID;
    SPH_TRY(ensure_params(c));
    SPH_CHECK_HIP(hipMemcpyAsync(c->mlp_params.p, params, NP * sizeof(float), hipMemcpyHostToDevice, c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(c->mlp_m.p, 0, NT * sizeof(float), c->stream));
    SPH_CHECK_HIP(hipMemsetAsync(c->mlp_v.p, 0, NT * sizeof(float), c->stream));
    c->adam_t = 0;
    SPH_TRY(pack((const float*)c->mlp_params.p, (MlpPacked*)c->mlp_packed.p, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    c->mlp_have = c->mlp_ready = true;
    return SPH_OK;
}

sph_status sph_h_get_params(sph_ctx* c, float* params)
{
    if (!c || !params) return SPH_ERR_INVALID;
    if (!c->mlp_have) return SPH_ERR_STATE;
    SPH_CHECK_HIP(hipMemcpyAsync(params, c->mlp_params.p, NP * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    SPH_CHECK_HIP(hipStreamSynchronize(c->stream));
    return SPH_OK;
}

sph_status sph_h_predict(sph_ctx* c, int on)
{
    if (!c || (on != 0 && on != 1)) return SPH_ERR_INVALID;
    if (on && !c->mlp_ready) return SPH_ERR_STATE;
    c->h_pred = on == 1;
    return SPH_OK;
}

}  // extern "C"
