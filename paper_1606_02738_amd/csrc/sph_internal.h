// Internal data layout of libsph_hip (gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph.h"

#define SPH_WAVE 64
#define SPH_MAX_LEAF 64          // particles per leaf cell (one wave of lanes)
#define SPH_NDIR 13              // axis directions between neighbouring cells
#define SPH_MAX_DEPTH 16         // octree levels below the top grid

// One periodic box ("domain") and its top-level cell grid.
struct DomainInfo {
    double L[3];      // box edges
    double s0[3];     // top-cell edges (>= largest H of the box)
    int n_top[3];     // top cells per dimension (>= 3)
    int top_offset;   // global index of the box's first top cell
    double pl_smax;   // particle lists: largest skin in the box (the top cells cover the
                      // largest list radius plus twice this)
    double pl_alpha;  // particle lists: fraction of the skins and growth allowances the
                      // box's top cells can hold (1 unless the box is small against them)
};

// Feature grid of one box for the learned H predictor: G cells per axis,
// scale = G / L, mean spacing (V/n)^(1/3), mean count per cell, offset of
// the box's counts in the shared count array.
struct FeatGrid {
    int G[3];
    int pad;
    double scale[3];
    double sbox;
    double nbar;
    long long off;
};

// Octree cell.  Children of a cell are contiguous in the node array.
struct Node {
    uint64_t key_lo;  // first Morton key of the cell
    int begin, count; // particle range (Morton order)
    int first_child;  // -1 for a leaf
    int n_child;
    int level, domain;
    int leaf;         // leaf id or -1
    int top;          // global top-cell index
    double lo[3], hi[3];   // tight bounding box of the particles
    double hmax;           // largest H in the cell (subtree)
    double hmin;           // smallest H in the cell
    double c_lo[3], c_sz[3];  // geometric cell corner and edge lengths
    int merged;            // 1: run of sibling octants merged into one leaf
    int pad;
};

// Compact copy of a cell for the list walk: bounding box rounded outward to
// float, children, particle count and leaf id.
struct WNode {
    float lo[3], hi[3];
    int first_child;
    int next;         // node after this subtree in depth-first order (-1: end of the top cell)
    int count;
    int leaf;
    float hl;         // upper bound of the list radii of the leaves below (symmetric lists)
    int pad;          // children (0 for a leaf cell)
};

// Neighbour-cell list entry of leaf A: leaf B, periodic image and the
// sort direction to use for the pair.  A's list holds every leaf B whose
// bounding box (image) lies closer than h_A (the radius the list was built
// for), i.e. the cells the density gather of A needs.
// Bytes per particle the one-pass list walk may hold in per-leaf slots, and
// in the shared overflow chunks of 64 entries that leaves with more entries
// than their slot continue into (leaves that find no free chunk are walked
// a second time).
#define SPH_WALK_SLOT_BYTES 64
#define SPH_WALK_OVF_BYTES 16

struct ListEntry {
    int B;
    int code;         // shift index (0..26) | dir << 8
    double dist;      // box-to-box distance, computed in a canonical order so
                      // that the entries (A,B) and (B,A) hold the same bits
};

// Relative margin added to a cell's largest H when its list is built, so
// that small growth of H during the iteration needs no new list.
#define SPH_LIST_SKIN 0.05
// The same margin of a particle's own list radius (particle lists); below
// SPH_LIST_SKIN, so the cell lists hold every pair the particle lists need.
#define SPH_PLIST_SKIN 0.02
// Largest growth factor of a particle's list radius (the growth of its H
// predicted over the lists' lifetime, see k_plist_ext).
#define SPH_PLIST_GROWTH_MAX 1.5

// Smallest residual tolerance |rho H^3 - C| / C of the FP32 modes (the
// sums' own resolution).  The converged H then differs from the exact root by
// about tol / (3 Omega), and rho by tol |1 - 1/Omega| (Omega reaches ~0.15 in
// the clustered box), so the compensated mode keeps rho within a few 1e-6.
#define SPH_FP32C_TOL_MIN 2.5e-7
#define SPH_FP32_TOL_MIN 2e-6

// Largest leaf extent / smallest H of the leaf in the FP32 modes.
#define SPH_FP32_EXTENT_RATIO 16.0

__host__ __device__ inline int shift_index(int sx, int sy, int sz) { return (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1); }

// The 13 directions between a cell and its 26 neighbours (one per +/- pair).
__host__ __device__ inline void sph_dir(int k, double* d)
{
    const int t[13][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1},
                          {0, 1, 1}, {0, 1, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    double n = sqrt((double)(t[k][0] * t[k][0] + t[k][1] * t[k][1] + t[k][2] * t[k][2]));
    d[0] = t[k][0] / n; d[1] = t[k][1] / n; d[2] = t[k][2] / n;
}

// Device-side error / event flags (bit mask in ctx->d_flags).
enum {
    FLAG_INVALID = 1,      // NaN / non-positive / out-of-box input
    FLAG_RELIST = 2,       // some H grew beyond the radius the lists were built for
    FLAG_REBUILD = 4,      // some H grew beyond the top-cell edge
    FLAG_BOX_SMALL = 8,    // some H reached the box limit with f < 0
    FLAG_STALE = 16,       // a leaf's H plus the displacement margin left its list radius
};

// Slots of the int[64] flags buffer.
enum { FI_FLAGS = 0, FI_SCRATCH = 8, FI_NCHILD = 9, FI_NLEAVES = 10, FI_NLIST = 11, FI_GATE = 12, FI_MAXLEAF = 13, FI_MAXLIST = 14, FI_PLROWS = 15, FI_WOVF = 16,
       FI_WINC = 17, FI_NCHUNK = 18, FI_NFLAGS = 64 };

// Counters written by kernels (device, int64).
enum { CNT_UNCONV = 0, CNT_NDENS = 1, CNT_NFORCE = 2, CNT_NPLIST = 3, CNT_DEVAL = 5, CNT_NPAIR = 6, CNT_NDENS_F = 7, CNT_GSWEEPS = 8, CNT_UHIST = 9, CNT_N = 16 };
// Task queues of the persistent force kernels, behind the counters above:
// XQ_N = 8, one per XCD, XQ_STRIDE counters (128 bytes) apart.  (64 queues,
// 8 per XCD, made the force loop slower.)
enum { XQ_N = 8, XQ_STRIDE = 16, XQ_FORCE = CNT_N };
// Particle lists: particles whose list failed the validity test of the last
// drift, by reason (moved beyond the skin, H beyond the list radius).
enum { CNT_STALE_MOVED = CNT_N + XQ_N * XQ_STRIDE, CNT_STALE_GROWN,
       // running totals of the force stage's counts since sph_create
       CNT_NFORCE_SUM, CNT_NDENS_SUM, CNT_FORCE_CALLS, CNT_ALLOC };

// Leaf arrays (device SoA).
struct LeafArrays {
    int* begin;
    int* count;
    double* origin;   // 3 per leaf: reference point of the cell-relative coordinates
    double* lo;       // 3 per leaf
    double* hi;       // 3 per leaf
    double* hlist;    // radius the neighbour lists were built for
    int* dom;
    int* list_off;    // n_leaves + 1
    int* active;      // leaf has unconverged particles
    int* sorted;      // 1 if the per-direction sort is valid
};

// Kernel-side view of the per-box constants and physics parameters.
struct PhysParams {
    double gamma;
    double C_fac;     // (kernel_gamma * eta)^3
    double h_tol;
};

// Workgroups are dealt to the 8 XCDs of the chip round-robin (workgroup b
// runs on XCD b mod 8), and each XCD has its own L2.  The logical block
// index below gives every XCD one contiguous range of blocks, so
// neighbouring leaves (Morton order) share an L2.  A bijection on [0, G).
__device__ inline int xcd_block(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (b >> 3);
}

// Device helpers shared by the kernels.
template <typename T> struct vec4;
template <> struct vec4<float> { typedef float4 type; };
template <> struct vec4<double> { typedef double4 type; };

__device__ inline uint64_t double_as_u64(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ inline double u64_as_double(uint64_t v) { return __longlong_as_double((long long)v); }

// Positive doubles order like their bit patterns: atomic max via integer max.
__device__ inline void atomic_max_pos_double(double* addr, double v)
{
    atomicMax((unsigned long long*)addr, (unsigned long long)double_as_u64(v));
}
