// Internal header of the gfx950 SPH + octree library: device helpers, the device-side
// workspace layout and the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned long long u64;
typedef unsigned int u32;
typedef unsigned short u16;

// ---------------------------------------------------------------------------------------
// Sticky device error bits (read back by sph_sync / synchronous calls).
enum : u32 {
    ERR_NONFINITE = 1u,      // non-finite position, velocity or energy
    ERR_NONPOSITIVE = 2u,    // h <= 0 or m <= 0
    ERR_NBR_CAP = 4u,        // a particle has more neighbours than nbr_capacity
    ERR_WALK_STACK = 8u,     // tree-walk stack or candidate list overflow
    ERR_NODE_CAP = 16u,      // octree node capacity exceeded
    ERR_GRAV_LIST = 32u,     // gravity walk stack overflow
    ERR_UNION_CAP = 64u,     // a walk group's source union exceeds UNION_MAX particles
};

// List entries are 16-bit indices into their group's source union, so a union holds at most
// this many particles (unions of a few thousand are typical).
constexpr int UNION_MAX = 65536;

constexpr int MAX_LEVEL = 21;   // 21 three-bit digits below the sentinel bit 63
constexpr double M_1_PI_D = 0.318309886183790671537767526745028724;

// Counter slots of the gravity pass's term counts, one 128-byte line each.
constexpr int GRAV_SLOTS = 64;

// Control block living in device memory.
struct DevCtl {
    u32 err;
    int n_nodes;
    int n_leaves;
    int nbr_max;                  // largest neighbour count seen (for overflow reports)
    int n_groups;                 // target groups
    int level_count[24];          // nodes per level
    int level_off[24];            // exclusive prefix of level_count
    u64 box_enc[512 * 6];         // per segment: ordered-integer min x,y,z then max x,y,z
    double box[512 * 6];          // decoded per-segment box lo.xyz, hi.xyz
    double scale[512];            // 2^B / L per segment (0 when L == 0)
    double side[512];             // L (root cell side) per segment
    double diag[16];              // step diagnostics
    double seg_dt[512];           // step size of each segment (read by the kick kernels)
    u64 dtb_enc[512];             // per segment: ordered-integer min of the time-step bound
    // last quadrupole gravity pass: particle-cell terms ([s][0]) and particle-particle terms
    // ([s][1], each target's own pair included) evaluated, summed over the slots s; a group
    // adds its counts to slot (group % GRAV_SLOTS), so the atomics spread over 64 lines
    u64 grav_cnt[GRAV_SLOTS][16];
    int skip_phi;                 // nonzero: the gravity passes leave phi unevaluated
};

// Device pointers of one context.  All arrays are carved out of the caller's workspace.
struct DevPtrs {
    DevCtl* ctl;
    // sort
    u64 *key_a, *key_b;           // n_cap
    u32 *val_a, *val_b;           // n_cap
    u32* rs_hist;                 // 256 * rs_blocks_cap
    u32* rs_dtot;                 // 256 digit totals of the current pass
    void* scan_tmp;               // 8 * scan_blocks_cap (u64)
    // Morton-ordered particle data (SoA FP64)
    double *x, *y, *z, *vx, *vy, *vz, *m, *h, *u;
    double *vpx, *vpy, *vpz, *up;  // predictors (step)
    double *ax, *ay, *az, *du;
    double *rho, *P, *cs, *hnext;
    double *gx, *gy, *gz, *phi;
    // second copies used while reordering between steps
    double *x2, *y2, *z2, *vx2, *vy2, *vz2, *m2, *h2, *u2, *vpx2, *vpy2, *vpz2, *up2;
    u32* id;                      // caller index of each Morton position
    u32* id2;
    double4* pos4;                // x, y, z, h (Morton order)
    double4* vel4;                // vx(pred), vy, vz, m
    double4* thr4;                // rho, P/rho^2, c, u
    float4* thrf;                 // FP32 copy for the compensated path: rho, P/rho^2, c, h
    // tree
    signed char* lcp;             // n_cap + 1: shared leading digits with the previous key
    unsigned char* lvl;           // n_cap: leaf level of each sorted position
    u64* scan_in;                 // n_cap + 1: (nodes at position << 32) | leaf start
    u64* scan_out;                // n_cap + 1
    int* leaf_start;              // n_cap + 1 (sorted position of each leaf, then n)
    int* leaf_pre;                // n_cap: pre-order node of each leaf
    unsigned char* pre_level;     // node_cap (pre-order)
    unsigned char* pre_leaf;      // node_cap
    int* pre_start;               // node_cap
    int* pre_to_bfs;              // node_cap
    int* bfs_to_pre;              // node_cap
    int* lsort_hist;              // 24 * lsort_tiles_cap
    int4* topo;                   // node_cap: {first, count, level, is_leaf}
    int* parent;                  // node_cap
    int* counter;                 // node_cap
    int2* range;                  // node_cap: {start, count} in sorted order
    double4* nbox_lo;             // node_cap: lo.xyz, hmax
    double4* nbox_hi;             // node_cap: hi.xyz, cell side
    double4* mom0;                // node_cap: M, com.xyz
    double4* mom1;                // node_cap: Ixx, Iyy, Izz, tr I
    double4* mom2;                // node_cap: Ixy, Ixz, Iyz, cell (bits; node-node gravity only)
    // groups and neighbour lists
    int4* group;                  // group_cap: {start, count, segment root rank (-1 = root), 0}
    u32* gflag;                   // n_cap + 1: 1 where a target group starts
    u32* gscan;                   // n_cap + 1
    u32* gsize;                   // n_cap + 1: size of the target group starting at a flagged position
    u16* nbr;                     // n_cap * nbr_cap: list slots, indices into the group's union
    int* nbr_cnt;                 // n_cap
    int* nbr_base;                // n_cap: group whose lists hold the particle (-1 = none)
    int* uni;                     // n_cap * nbr_cap: per group, particles of its source union
    int* ucnt;                    // group_cap: size of each group's union
    // seg / chunk tables
    int4* chunk;                  // chunk_cap: {begin, end, seg, 0} in caller/Morton order
    int* seg_root_rank;           // seg_cap: rank of the segment among non-empty segments
    // diagnostics partials
    double* diag_part;            // 16 * diag_blocks
    // CSR export
    int64_t* csr_tmp;             // n_cap + 1 (counts / offsets in caller order)
};

struct Dims {
    int n;            // particles
    int n_seg;        // 1 = one set
    int batched;      // n_seg > 1
    int leaf_size;
    int group_size;
    int nbr_cap;
    int group_grid;   // grid (multiple of 8) of the one-wave per-group kernels
    int pair_grid;    // the same for the four-wave pair kernels (density, forces)
    int n_chunks;
    int node_cap;
    int min_level;    // 3 when batched, else 0
    int curve;        // 0 Morton, 1 Hilbert keys
    int mass_moments; // node masses and moments are built (only the gravity kernels read them)
};

// Key quantisation of one coordinate (Sec. 2.1): one subtraction, one multiplication, then
// truncation into 0 .. top (the cell index inside the cubic root cell at the finest level).
__device__ __forceinline__ u32 quantise(double x, double lo, double S, u32 top) {
    double t = (x - lo) * S;
    if (!(t > 0.0)) return 0u;
    if (t >= (double)top) return top;
    return (u32)t;
}

// ---------------------------------------------------------------------------------------
// Wave helpers (wave64 on gfx950)

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}
// A value every active lane holds (a wave reduction's result) moved to scalar registers, so
// that it costs no vector registers where it is only read.
__device__ __forceinline__ double uniform_d(double v) {
    const u64 b = (u64)__double_as_longlong(v);
    const u32 lo = __builtin_amdgcn_readfirstlane((u32)b), hi = __builtin_amdgcn_readfirstlane((u32)(b >> 32));
    return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}

// Sum over the 64/gsz lanes that serve one target (lanes t, t+gsz, ...), fixed order.
__device__ __forceinline__ double lanes_sum_d(double v, int gsz) {
    for (int off = gsz; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Persistent, XCD-aware loop over groups.  Workgroups are dispatched round-robin over the
// 8 XCDs (blockIdx % 8); the workgroups of one XCD take one contiguous eighth of the groups,
// so neighbouring groups -- which read the same neighbour particles -- share an L2.
__device__ __forceinline__ void group_range(int n_groups, int& g0, int& g1, int& step) {
    const int nx = 8;
    const int xcd = (int)(blockIdx.x % nx), j = (int)(blockIdx.x / nx);
    step = (int)(gridDim.x / nx);
    const int chunk = (n_groups + nx - 1) / nx;
    g0 = xcd * chunk + j;
    g1 = min(n_groups, (xcd + 1) * chunk);
}

// Ordered-integer encoding of doubles for exact atomic min/max.
__device__ __forceinline__ u64 enc_double(double d) {
    u64 b = (u64)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dec_double(u64 e) {
    u64 b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ void set_err(DevCtl* ctl, u32 bits) { atomicOr(&ctl->err, bits); }

// Block-wide min/max of a chunk's positions (blockDim.x a multiple of 64, at most 1024),
// merged into the segment's box with order-independent atomics on the encoded values.
__device__ __forceinline__ void box_block_merge(DevCtl* ctl, int seg, double lo[3], double hi[3], bool any) {
    __shared__ double red[16][6];
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = wave_min(lo[c]);
        hi[c] = wave_max(hi[c]);
    }
    if (lane_id() == 0) {
        for (int c = 0; c < 3; ++c) {
            red[w][c] = lo[c];
            red[w][3 + c] = hi[c];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6 && any) {
        const int c = threadIdx.x;
        double v = red[0][c];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) v = (c < 3) ? fmin(v, red[k][c]) : fmax(v, red[k][c]);
        u64* slot = &ctl->box_enc[6 * seg + c];
        if (c < 3) atomicMin(slot, enc_double(v));
        else atomicMax(slot, enc_double(v));
    }
}

// Leading equal 3-bit digits (0..21) of two keys below the sentinel.
__device__ __forceinline__ int lcp_digits(u64 a, u64 b) {
    u64 x = (a ^ b) & 0x7fffffffffffffffull;
    if (x == 0) return MAX_LEVEL;
    return (__clzll(x) - 1) / 3;
}

// ---------------------------------------------------------------------------------------
// M4 cubic spline (support 2h): W = w(q) / (pi h^3), grad_a W_ab = r_ab g(q) / (pi h^5),
// g = w'(q) / q; and compensated FP32 accumulators.  Both pieces are evaluated and one is
// selected, so a wavefront never splits on q.

__device__ __forceinline__ double m4_w(double q) {
    const double t = fmax(2.0 - q, 0.0);
    const double wo = 0.25 * (t * t * t);
    const double wi = fma(q * q, fma(0.75, q, -1.5), 1.0);
    return q < 1.0 ? wi : wo;
}
// g(q) given 1/q (unused, and may be inf or NaN, for q < 1)
__device__ __forceinline__ double m4_g(double q, double inv_q) {
    const double t = fmax(2.0 - q, 0.0);
    const double go = -0.75 * (t * t) * inv_q;
    const double gi = fma(2.25, q, -3.0);
    return q < 1.0 ? gi : go;
}
__device__ __forceinline__ float m4_wf(float q) {
    const float t = fmaxf(2.0f - q, 0.0f);
    const float wo = 0.25f * (t * t * t);
    const float wi = fmaf(q * q, fmaf(0.75f, q, -1.5f), 1.0f);
    return q < 1.0f ? wi : wo;
}
__device__ __forceinline__ float m4_gf(float q, float inv_q) {
    const float t = fmaxf(2.0f - q, 0.0f);
    const float go = -0.75f * (t * t) * inv_q;
    const float gi = fmaf(2.25f, q, -3.0f);
    return q < 1.0f ? gi : go;
}

// FP64 reciprocal and square root for the pair sums, from the hardware estimates refined
// by Newton-Raphson steps (reciprocal: r <- r + r (1 - x r), twice) and by one Goldschmidt
// step plus one Newton correction (square root); a few ulp, not correctly rounded.
// rcp_nr: x positive and normal.  sqrt_nr: a >= 0 (0 gives 0).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
// 1/sqrt(a) for a positive and normal: two Newton steps y <- y (3/2 - a y^2 / 2).
__device__ __forceinline__ double rsq_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}
// One Newton step only: the hardware estimate (~5e-8 relative) refined to ~4e-15, for sums
// whose own approximation error is far larger (tree gravity).
__device__ __forceinline__ double rsq_nr1(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    return y * fma(-0.5 * a * y, y, 1.5);
}
__device__ __forceinline__ double sqrt_nr(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double r = a * y, h = 0.5 * y;
    const double e = fma(-r, h, 0.5);
    r = fma(r, e, r);
    h = fma(h, e, h);
    const double d = fma(-r, r, a);
    r = fma(d, h, r);
    return a > 0.0 ? r : 0.0;
}
// sqrt(a) and 1/sqrt(a) together, a >= 0: the Goldschmidt step of sqrt_nr refines both;
// the inverse to about 1e-14 relative (a == 0 gives sqrt 0 and a non-finite inverse).
__device__ __forceinline__ double sqrt_rsq_nr(double a, double& inv) {
    const double y = __builtin_amdgcn_rsq(a);
    double r = a * y, h = 0.5 * y;
    const double e = fma(-r, h, 0.5);
    r = fma(r, e, r);
    h = fma(h, e, h);
    const double d = fma(-r, r, a);
    r = fma(d, h, r);
    inv = 2.0 * h;
    return a > 0.0 ? r : 0.0;
}

// Kahan accumulator (explicit operation order; the library is built without floating-point
// contraction, so it is not fused).
struct Kahan {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};


// ---------------------------------------------------------------------------------------
// Launchers (defined in the .hip files)

// k_build.hip
void launch_fill_u32(hipStream_t s, u32* p, u32 v, int n);
void launch_fill_i32(hipStream_t s, int* p, int v, int n);
void launch_bbox(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* x, const double* y,
                 const double* z, const u32* perm_or_null);
void launch_set_box(hipStream_t s, const DevPtrs& d, const Dims& dm, int from_host_box);
void launch_keys(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* x, const double* y,
                 const double* z, const double* vx, const double* vy, const double* vz, const double* m,
                 const double* h, const double* u, u64* keys_out_caller, int caller_order);
void radix_sort(hipStream_t s, const DevPtrs& d, int n);
void scan_u64(hipStream_t s, const u64* in, u64* out, int n, void* tmp);
void scan_u32_total(hipStream_t s, const u32* in, u32* out, int n, void* tmp);
void launch_gather_input(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* x, const double* y,
                         const double* z, const double* vx, const double* vy, const double* vz, const double* m,
                         const double* h, const double* u, int64_t* order_out);
// k_tree.hip
void build_octree(hipStream_t s, const DevPtrs& d, const Dims& dm);
void launch_tree_export(hipStream_t s, const DevPtrs& d, const Dims& dm, u64* key, int32_t* level,
                        int32_t* leaf, int64_t* start, int64_t* count);
// k_walk.hip
// neighbour lists + density, EOS and h_next (u_eos: the energy the EOS uses)
void launch_nbr_lists(hipStream_t s, const DevPtrs& d, const Dims& dm);
void launch_density(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double gamma, double h_coeff,
                    const double* u_eos, int kinetic_in_u);
void launch_csr_count(hipStream_t s, const DevPtrs& d, const Dims& dm, int64_t* counts_caller);
void scan_i64_inplace(hipStream_t s, int64_t* a, int n, void* tmp);
void launch_csr_fill(hipStream_t s, const DevPtrs& d, const Dims& dm, const int64_t* offsets, int32_t* idx);
// k_sph.hip
void launch_thermo_from_caller(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* rho,
                               const double* P, const double* cs);
void launch_forces(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double alpha, double beta,
                  double eps_av, int thermokinetic);
// k_grav.hip
void launch_gravity(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double G, double eps,
                    double theta, int accumulate, int thermokinetic);
void launch_fmm(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double G, double eps, double theta,
                int accumulate, int thermokinetic);
// k_step.hip
void launch_scatter_caller(hipStream_t s, const DevPtrs& d, int n, const double* src, double* dst);
void launch_fill_zero(hipStream_t s, int n, double* dst);
void launch_gather_caller(hipStream_t s, const DevPtrs& d, int n, const double* src_caller, double* dst);
void launch_box_init(hipStream_t s, const DevPtrs& d, const Dims& dm);
void launch_kick_drift(hipStream_t s, const DevPtrs& d, const Dims& dm, bool pre_kick, int adaptive_h);
void launch_step_keys(hipStream_t s, const DevPtrs& d, const Dims& dm);
void launch_step_permute(hipStream_t s, const DevPtrs& d, int n);
void launch_kick(hipStream_t s, const DevPtrs& d, const Dims& dm, int adaptive_h);
void launch_set_hnext(hipStream_t s, const DevPtrs& d, int n);
void launch_diag(hipStream_t s, const DevPtrs& d, const Dims& dm, int with_phi, int kinetic_in_u, double eps_grav);
void launch_write_back(hipStream_t s, const DevPtrs& d, int n, double* x, double* y, double* z, double* vx,
                       double* vy, double* vz, double* h, double* u, double* ax, double* ay, double* az,
                       double* du, int kinetic_in_u);
void launch_dt_bound(hipStream_t s, const DevPtrs& d, const Dims& dm, double eps_grav);
void launch_resident_export(hipStream_t s, const DevPtrs& d, int n, u64* keys_caller, int64_t* order);
void launch_add_kinetic(hipStream_t s, const DevPtrs& d, int n);
void launch_load_accel(hipStream_t s, const DevPtrs& d, int n, const double* ax, const double* ay,
                       const double* az, const double* du);
