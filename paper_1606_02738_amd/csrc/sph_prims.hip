// Device primitives: exclusive scan of int32 and a stable LSD radix sort of
// (uint64 key, uint32 value) pairs.  Written for wave64 (gfx950).
#include "sph_ctx.h"

#define SCAN_T 256
#define SCAN_ITEMS 4
#define SCAN_BLOCK (SCAN_T * SCAN_ITEMS)

// Exclusive scan of one 1024-element tile per workgroup; the tile total goes
// to block_sums[blockIdx.x].  Each thread loads its items before writing, so
// in == out is allowed.
__global__ __launch_bounds__(SCAN_T) void k_scan_block(const int* in, int* out, int n, int* block_sums)
{
    __shared__ int wsum[SCAN_T / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long base = (long)blockIdx.x * SCAN_BLOCK + (long)tid * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        s += v[k];
    }
    int incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int wprefix = 0;
    for (int q = 0; q < w; q++) wprefix += wsum[q];
    int excl = wprefix + incl - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long idx = base + k;
        if (idx < n) out[idx] = excl;
        excl += v[k];
    }
    if (tid == SCAN_T - 1 && block_sums) block_sums[blockIdx.x] = wprefix + incl;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_add(int* out, int n, const int* offs)
{
    const long base = (long)blockIdx.x * SCAN_BLOCK + (long)threadIdx.x * SCAN_ITEMS;
    const int o = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long idx = base + k;
        if (idx < n) out[idx] += o;
    }
}

static sph_status scan_rec(sph_ctx* c, const int* in, int* out, int n, int* d_total, int* tmp, long tmp_left)
{
    const int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb <= 1) {
        k_scan_block<<<1, SCAN_T, 0, c->stream>>>(in, out, n, d_total);
        SPH_CHECK_LAUNCH();
        return SPH_OK;
    }
    if (tmp_left < nb) return SPH_ERR_WORKSPACE;
    int* bs = tmp;
    k_scan_block<<<nb, SCAN_T, 0, c->stream>>>(in, out, n, bs);
    SPH_CHECK_LAUNCH();
    SPH_TRY(scan_rec(c, bs, bs, nb, d_total, tmp + nb, tmp_left - nb));
    k_scan_add<<<nb, SCAN_T, 0, c->stream>>>(out, n, bs);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

sph_status scan_exclusive(sph_ctx* c, const int* in, int* out, int n, int* d_total)
{
    if (n <= 0) {
        SPH_CHECK_HIP(hipMemsetAsync(d_total, 0, sizeof(int), c->stream));
        return SPH_OK;
    }
    long need = (long)n / SCAN_BLOCK + 64;
    SPH_TRY(buf_ensure(c->scan_tmp, need * sizeof(int)));
    return scan_rec(c, in, out, n, d_total, (int*)c->scan_tmp.p, need);
}

// ---------------------------------------------------------------------------
// Radix sort: 8-bit digits.  A workgroup owns a tile of RS_TILE keys; wave w
// of the workgroup owns the contiguous quarter w of the tile, and lane l of
// the wave holds keys r*64 + l of that quarter (r = 0..RS_ITEMS-1), so rounds
// visit the quarter in order.  The per-digit global offsets come from an
// exclusive scan of the digit-major [256][n_tiles] histogram.
// ---------------------------------------------------------------------------
#define RS_WAVES 4
#define RS_ITEMS 16
#define RS_TILE (64 * RS_WAVES * RS_ITEMS)

__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t* __restrict__ keys, int n, int shift, int* hist, int nb)
{
    __shared__ int h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const long base = (long)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_TILE / 256; k++) {
        long idx = base + (long)k * 256 + tid;
        if (idx < n) atomicAdd(&h[(int)((keys[idx] >> shift) & 255u)], 1);
    }
    __syncthreads();
    hist[(long)tid * nb + blockIdx.x] = h[tid];
}

// The tile's keys are ranked stably by digit into LDS (local order: wave,
// round, lane, i.e. input order within each digit), then written out in
// that order: consecutive lanes write consecutive positions of one digit's
// run, so the stores coalesce into runs of ~RS_TILE / 256 keys.
__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int n,
                                                    int shift, const int* __restrict__ offs, int nb)
{
    __shared__ int wcount[RS_WAVES][256];
    __shared__ int wbase[RS_WAVES][256];
    __shared__ int gshift[256];  // global position - local position, per digit
    __shared__ int wsum[RS_WAVES];
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[RS_TILE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = tid; q < RS_WAVES * 256; q += 256) (&wcount[0][0])[q] = 0;
    __syncthreads();
    const long tile = (long)blockIdx.x * RS_TILE;
    const long wstart = tile + (long)w * 64 * RS_ITEMS;
    uint64_t k[RS_ITEMS];
    uint32_t v[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        long idx = wstart + (long)r * 64 + lane;
        if (idx < n) {
            k[r] = kin[idx];
            v[r] = vin[idx];
            atomicAdd(&wcount[w][(int)((k[r] >> shift) & 255u)], 1);
        } else {
            k[r] = 0;
            v[r] = 0;
        }
    }
    __syncthreads();
    {
        // local start of digit d: exclusive scan over the digits of the
        // tile's counts (one digit per thread: wave scans, then wave sums)
        const int d = tid;
        int cnt = 0;
        for (int q = 0; q < RS_WAVES; q++) cnt += wcount[q][d];
        int inc = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(inc, off);
            if (lane >= off) inc += t;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int start = inc - cnt;
        for (int q = 0; q < w; q++) start += wsum[q];
        gshift[d] = offs[(long)d * nb + blockIdx.x] - start;
        int run = start;
        for (int q = 0; q < RS_WAVES; q++) {
            wbase[q][d] = run;
            run += wcount[q][d];
        }
    }
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        const long idx = wstart + (long)r * 64 + lane;
        const bool valid = idx < n;
        const int d = (int)((k[r] >> shift) & 255u);
        unsigned long long mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1;
            unsigned long long bb = __ballot(valid && bit);
            mask &= bit ? bb : ~bb;
        }
        const int rank = __popcll(mask & lt);
        int base = 0;
        if (valid) base = wbase[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wbase[w][d] = base + __popcll(mask);
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            sk[base + rank] = k[r];
            sv[base + rank] = v[r];
        }
    }
    __syncthreads();
    const int in_tile = (int)min((long)RS_TILE, (long)n - tile);
    for (int e = tid; e < in_tile; e += 256) {
        const uint64_t kk = sk[e];
        const int pos = gshift[(int)((kk >> shift) & 255u)] + e;
        kout[pos] = kk;
        vout[pos] = sv[e];
    }
}

sph_status radix_sort(sph_ctx* c, int n, int bits, DevBuf* kb, DevBuf* vb, int* res_idx)
{
    int cur = 0;
    if (n > 1) {
        const int nb = (n + RS_TILE - 1) / RS_TILE;
        SPH_TRY(buf_ensure(c->rs_hist, (size_t)256 * nb * sizeof(int) + 64));
        int* hist = (int*)c->rs_hist.p;
        int* total = (int*)c->flags.p + FI_SCRATCH;
        for (int shift = 0; shift < bits; shift += 8) {
            uint64_t* kin = (uint64_t*)kb[cur].p;
            uint32_t* vin = (uint32_t*)vb[cur].p;
            uint64_t* kout = (uint64_t*)kb[cur ^ 1].p;
            uint32_t* vout = (uint32_t*)vb[cur ^ 1].p;
            k_rs_hist<<<nb, 256, 0, c->stream>>>(kin, n, shift, hist, nb);
            SPH_CHECK_LAUNCH();
            SPH_TRY(scan_exclusive(c, hist, hist, 256 * nb, total));
            k_rs_scatter<<<nb, 256, 0, c->stream>>>(kin, vin, kout, vout, n, shift, hist, nb);
            SPH_CHECK_LAUNCH();
            cur ^= 1;
        }
    }
    *res_idx = cur;
    return SPH_OK;
}
