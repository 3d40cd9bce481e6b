// Keys, sort and snapshot (Sec. 2.1 "Tree topology" of arXiv:2007.03097, Fig. 1).
//
//  * k_bbox      exact per-segment bounding box (ordered-integer atomics, order independent)
//  * k_keys      quantise to B bits inside the cubic root cell, interleave (x lowest) or
//                Hilbert index, sentinel bit 63, segment number in bits 54..62 for
//                segmented sets
//  * radix sort  stable LSD, 8 passes of 8-bit digits over (key, caller index); stability
//                plus an identity initial order gives the (key, ID) order of the paper
//  * gather      caller-order input -> key-ordered SoA + AoS records
#include "common.h"

// ---------------------------------------------------------------------------------------
// fills
__global__ void k_fill_u32(u32* p, u32 v, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int* p, int v, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
static int grid_for(int n, int bs = 256, int cap = 4096) {
    int g = (n + bs - 1) / bs;
    return g < 1 ? 1 : (g > cap ? cap : g);
}
void launch_fill_u32(hipStream_t s, u32* p, u32 v, int n) {
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
}
void launch_fill_i32(hipStream_t s, int* p, int v, int n) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
}

// ---------------------------------------------------------------------------------------
// bounding box per segment.  The chunk table splits [0, n) into pieces that never cross a
// segment boundary; one block reduces a chunk and folds it into the segment's box with
// exact atomic min/max on an order-preserving integer encoding.
__global__ void k_box_init(DevCtl* ctl, int n_seg) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_seg) {
        for (int c = 0; c < 3; ++c) {
            ctl->box_enc[6 * s + c] = ~0ull;
            ctl->box_enc[6 * s + 3 + c] = 0ull;
        }
    }
}

__global__ void __launch_bounds__(256) k_bbox(DevCtl* ctl, const int4* chunk, const double* __restrict__ x,
                                               const double* __restrict__ y, const double* __restrict__ z) {
    const int4 ch = chunk[blockIdx.x];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = ch.x + threadIdx.x; i < ch.y; i += blockDim.x) {
        double v[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], v[c]);
            hi[c] = fmax(hi[c], v[c]);
        }
    }
    box_block_merge(ctl, ch.z, lo, hi, ch.y > ch.x);
}

void launch_box_init(hipStream_t s, const DevPtrs& d, const Dims& dm) {
    hipLaunchKernelGGL(k_box_init, dim3((dm.n_seg + 255) / 256), dim3(256), 0, s, d.ctl, dm.n_seg);
}

void launch_bbox(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* x, const double* y,
                 const double* z, const u32*) {
    hipLaunchKernelGGL(k_box_init, dim3((dm.n_seg + 255) / 256), dim3(256), 0, s, d.ctl, dm.n_seg);
    if (dm.n_chunks > 0) hipLaunchKernelGGL(k_bbox, dim3(dm.n_chunks), dim3(256), 0, s, d.ctl, d.chunk, x, y, z);
}

// Decode the boxes (unless the caller supplied them) and derive L and S = 2^B / L.
__global__ void k_set_box(DevCtl* ctl, int n_seg, int bits, int from_host) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    if (!from_host)
        for (int c = 0; c < 6; ++c) ctl->box[6 * s + c] = dec_double(ctl->box_enc[6 * s + c]);
    double L = 0.0;
    for (int c = 0; c < 3; ++c) {
        double e = ctl->box[6 * s + 3 + c] - ctl->box[6 * s + c];
        if (e > L) L = e;
    }
    double S = 0.0;
    if (L > 0.0) {
        S = (double)(1u << bits) / L;   // one IEEE division
        if (!isfinite(S)) S = 0.0;
    }
    ctl->scale[s] = S;
    ctl->side[s] = L;
}

void launch_set_box(hipStream_t s, const DevPtrs& d, const Dims& dm, int from_host_box) {
    hipLaunchKernelGGL(k_set_box, dim3((dm.n_seg + 255) / 256), dim3(256), 0, s, d.ctl, dm.n_seg,
                       dm.batched ? 18 : 21, from_host_box);
}

// ---------------------------------------------------------------------------------------
// keys
__device__ __forceinline__ u64 spread3(u32 v) {
    u64 x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Hilbert index of grid cell (x, y, z) on a 2^bits grid: Skilling's transposition
// (J. Skilling, AIP Conf. Proc. 707, 381 (2004)) unrolled for three axes, then one 3-bit
// digit per level with x in its high bit.
__device__ __forceinline__ u64 hilbert3(u32 x, u32 y, u32 z, int bits) {
    const u32 top = 1u << (bits - 1);
    for (u32 q = top; q > 1u; q >>= 1) {
        const u32 low = q - 1u;
        if (x & q) x ^= low;
        if (y & q) {
            x ^= low;
        } else {
            const u32 t = (x ^ y) & low;
            x ^= t;
            y ^= t;
        }
        if (z & q) {
            x ^= low;
        } else {
            const u32 t = (x ^ z) & low;
            x ^= t;
            z ^= t;
        }
    }
    y ^= x;
    z ^= y;
    u32 flip = 0u;
    for (u32 q = top; q > 1u; q >>= 1)
        if (z & q) flip ^= q - 1u;
    x ^= flip;
    y ^= flip;
    z ^= flip;
    return spread3(z) | (spread3(y) << 1) | (spread3(x) << 2);
}

__device__ __forceinline__ u64 make_key(double x, double y, double z, const double* lo, double S, int seg,
                                        int batched, int curve) {
    const int bits = batched ? 18 : 21;
    const u32 top = (1u << bits) - 1u;
    const u32 qx = quantise(x, lo[0], S, top), qy = quantise(y, lo[1], S, top), qz = quantise(z, lo[2], S, top);
    const u64 m = curve ? hilbert3(qx, qy, qz, bits) : (spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2));
    u64 k = (1ull << 63) | m;
    if (batched) k |= (u64)seg << 54;
    return k;
}

// Caller-order keys + input validation.  val = caller index (identity).
__global__ void __launch_bounds__(256) k_keys(DevCtl* ctl, const int4* chunk, int batched, int curve,
                                               const double* __restrict__ x, const double* __restrict__ y,
                                               const double* __restrict__ z, const double* __restrict__ vx,
                                               const double* __restrict__ vy, const double* __restrict__ vz,
                                               const double* __restrict__ m, const double* __restrict__ h,
                                               const double* __restrict__ u, u64* key, u32* val, u64* key_out) {
    const int4 ch = chunk[blockIdx.x];
    u32 bad = 0;
    for (int i = ch.x + threadIdx.x; i < ch.y; i += blockDim.x) {
        double px = x[i], py = y[i], pz = z[i];
        if (!isfinite(px) || !isfinite(py) || !isfinite(pz) || !isfinite(vx[i]) || !isfinite(vy[i]) ||
            !isfinite(vz[i]) || !isfinite(u[i]))
            bad |= ERR_NONFINITE;
        if (!(h[i] > 0.0) || !(m[i] > 0.0) || !isfinite(h[i]) || !isfinite(m[i])) bad |= ERR_NONPOSITIVE;
        u64 k = make_key(px, py, pz, ctl->box + 6 * ch.z, ctl->scale[ch.z], ch.z, batched, curve);
        key[i] = k;
        val[i] = (u32)i;
        if (key_out) key_out[i] = k;
    }
    if (bad) set_err(ctl, bad);
}

void launch_keys(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* x, const double* y,
                 const double* z, const double* vx, const double* vy, const double* vz, const double* m,
                 const double* h, const double* u, u64* keys_out_caller, int) {
    if (dm.n_chunks > 0)
        hipLaunchKernelGGL(k_keys, dim3(dm.n_chunks), dim3(256), 0, s, d.ctl, d.chunk, dm.batched, dm.curve, x, y, z, vx, vy,
                           vz, m, h, u, d.key_a, d.val_a, keys_out_caller);
}

// Step-loop keys: positions are in the previous key order; write the key at the caller
// index (so the sort input is again in caller order) and remember where each caller
// index sat.
// (the positions, velocities and energies it keys were checked for non-finite values by the
// kick-drift that wrote them)
__global__ void __launch_bounds__(256) k_step_keys(DevCtl* ctl, const int4* chunk, int batched, int curve,
                                                    const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const u32* __restrict__ id,
                                                    u64* key, u32* val) {
    const int4 ch = chunk[blockIdx.x];
    // the segment's box from the merged encodings, L and S = 2^B / L (one IEEE division);
    // the segment's first chunk publishes them for the tree build
    double box[6];
    for (int c = 0; c < 6; ++c) box[c] = dec_double(ctl->box_enc[6 * ch.z + c]);
    double L = 0.0;
    for (int c = 0; c < 3; ++c) L = fmax(L, box[3 + c] - box[c]);
    double S = 0.0;
    if (L > 0.0) {
        S = (double)(1u << (batched ? 18 : 21)) / L;
        if (!isfinite(S)) S = 0.0;
    }
    if (ch.w && threadIdx.x < 6) {
        ctl->box[6 * ch.z + threadIdx.x] = box[threadIdx.x];
        if (threadIdx.x == 0) {
            ctl->scale[ch.z] = S;
            ctl->side[ch.z] = L;
        }
    }
    for (int p = ch.x + threadIdx.x; p < ch.y; p += blockDim.x) {
        const double px = x[p], py = y[p], pz = z[p];
        const u32 i = id[p];  // keys go to caller order, so the stable sort orders ties by ID
        key[i] = make_key(px, py, pz, box, S, ch.z, batched, curve);
        val[i] = (u32)p;      // the sort carries each particle's current position
    }
}

void launch_step_keys(hipStream_t s, const DevPtrs& d, const Dims& dm) {
    if (dm.n_chunks > 0)
        hipLaunchKernelGGL(k_step_keys, dim3(dm.n_chunks), dim3(256), 0, s, d.ctl, d.chunk, dm.batched, dm.curve, d.x, d.y,
                           d.z, d.id, d.key_a, d.val_a);
}

// ---------------------------------------------------------------------------------------
// scans (exclusive), 256 threads x 8 items per block
constexpr int SC_THREADS = 256, SC_ITEMS = 8, SC_TILE = SC_THREADS * SC_ITEMS;

template <typename T>
__device__ T block_excl_scan(T v, T* total) {
    __shared__ T wsum[SC_THREADS / 64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    T off = 0, tot = 0;
    for (int k = 0; k < SC_THREADS / 64; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

template <typename T>
__global__ void __launch_bounds__(SC_THREADS) k_scan_reduce(const T* __restrict__ in, int n, T* sums) {
    const int base = blockIdx.x * SC_TILE + threadIdx.x * SC_ITEMS;
    T s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    T tot;
    block_excl_scan<T>(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SC_THREADS) k_scan_top(T* sums, int nb) {
    T carry = 0;
    for (int b0 = 0; b0 < nb; b0 += SC_TILE) {
        T v[SC_ITEMS];
        T s = 0;
#pragma unroll
        for (int k = 0; k < SC_ITEMS; ++k) {
            int i = b0 + threadIdx.x * SC_ITEMS + k;
            v[k] = (i < nb) ? sums[i] : (T)0;
            s += v[k];
        }
        T tot;
        T e = block_excl_scan<T>(s, &tot) + carry;
#pragma unroll
        for (int k = 0; k < SC_ITEMS; ++k) {
            int i = b0 + threadIdx.x * SC_ITEMS + k;
            if (i < nb) sums[i] = e;
            e += v[k];
        }
        carry += tot;
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(SC_THREADS) k_scan_down(const T* __restrict__ in, T* out, int n,
                                                          const T* __restrict__ sums, int write_total) {
    const int base = blockIdx.x * SC_TILE + threadIdx.x * SC_ITEMS;
    T v[SC_ITEMS];
    T s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : (T)0;
        s += v[k];
    }
    T tot;
    T e = block_excl_scan<T>(s, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        if (base + k < n) out[base + k] = e;
        if (write_total && base + k == n - 1) out[n] = e + v[k];
        e += v[k];
    }
}

// Down-sweep that first sums the block totals of the blocks before it (sums[] holds the
// totals of k_scan_reduce, not yet scanned): for up to SCAN_FUSE_MAX blocks this costs less
// than a separate one-workgroup launch over the totals.
constexpr int SCAN_FUSE_MAX = 4096;

template <typename T>
__global__ void __launch_bounds__(SC_THREADS) k_scan_down_fused(const T* __restrict__ in, T* out, int n,
                                                                const T* __restrict__ sums, int write_total) {
    T pre = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += SC_THREADS) pre += sums[i];
    T pre_tot;
    block_excl_scan<T>(pre, &pre_tot);
    const int base = blockIdx.x * SC_TILE + threadIdx.x * SC_ITEMS;
    T v[SC_ITEMS];
    T s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : (T)0;
        s += v[k];
    }
    T tot;
    T e = block_excl_scan<T>(s, &tot) + pre_tot;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        if (base + k < n) out[base + k] = e;
        if (write_total && base + k == n - 1) out[n] = e + v[k];
        e += v[k];
    }
}

template <typename T>
__global__ void k_zero_one(T* p) {
    if (threadIdx.x == 0) p[0] = (T)0;
}

template <typename T>
static void scan_impl(hipStream_t s, const T* in, T* out, int n, void* tmp, int write_total) {
    if (n <= 0) {
        if (write_total) hipLaunchKernelGGL(k_zero_one<T>, dim3(1), dim3(64), 0, s, out);
        return;
    }
    const int nb = (n + SC_TILE - 1) / SC_TILE;
    T* sums = (T*)tmp;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(SC_THREADS), 0, s, in, n, sums);
    if (nb <= SCAN_FUSE_MAX) {
        hipLaunchKernelGGL(k_scan_down_fused<T>, dim3(nb), dim3(SC_THREADS), 0, s, in, out, n, (const T*)sums,
                           write_total);
        return;
    }
    hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(SC_THREADS), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(SC_THREADS), 0, s, in, out, n, (const T*)sums, write_total);
}

// out[0..n) = exclusive scan, out[n] = total
void scan_u64(hipStream_t s, const u64* in, u64* out, int n, void* tmp) { scan_impl<u64>(s, in, out, n, tmp, 1); }
void scan_i64_inplace(hipStream_t s, int64_t* a, int n, void* tmp) {
    scan_impl<long long>(s, (const long long*)a, (long long*)a, n, tmp, 1);
}
static void scan_u32(hipStream_t s, u32* a, int n, void* tmp) { scan_impl<u32>(s, a, a, n, tmp, 0); }
void scan_u32_total(hipStream_t s, const u32* in, u32* out, int n, void* tmp) { scan_impl<u32>(s, in, out, n, tmp, 1); }

// ---------------------------------------------------------------------------------------
// LSD radix sort of (u64 key, u32 value), 8-bit digits, 8 passes.  Each block owns a tile
// of 2048 keys; wave w of the block owns keys [w*512, w*512 + 512) of the tile in 8 rounds
// of 64, so (wave, round, lane) order is index order and ranks are stable.
constexpr int RS_THREADS = 256, RS_ITEMS = 8, RS_TILE = RS_THREADS * RS_ITEMS, RS_WAVES = RS_THREADS / 64;

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const u64* __restrict__ key, int n, int shift, u32* hist,
                                                        int nb) {
    __shared__ u32 h[RS_WAVES][256];
    const int w = threadIdx.x >> 6, lane = lane_id();
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) (&h[0][0])[i] = 0;
    __syncthreads();
    const int base = blockIdx.x * RS_TILE + w * (64 * RS_ITEMS) + lane;
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        int i = base + r * 64;
        if (i < n) atomicAdd(&h[w][(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    u32 t = 0;
    for (int k = 0; k < RS_WAVES; ++k) t += h[k][threadIdx.x];
    hist[threadIdx.x * nb + blockIdx.x] = t;
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const u64* __restrict__ kin, const u32* __restrict__ vin,
                                                           u64* __restrict__ kout, u32* __restrict__ vout, int n,
                                                           int shift, const u32* __restrict__ offs, int nb,
                                                           const u32* __restrict__ digit_tot) {
    __shared__ u32 wcnt[RS_WAVES][256];
    __shared__ u32 woff[RS_WAVES][256];
    __shared__ u32 dbase[256];
    __shared__ u32 loff[256];
    __shared__ u32 gbase[256];
    __shared__ u64 sk[RS_TILE];
    __shared__ u32 sv[RS_TILE];
    const int w = threadIdx.x >> 6, lane = lane_id();
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
    {   // exclusive scan of the digit totals
        u32 tot;
        const u32 e = block_excl_scan<u32>(digit_tot[threadIdx.x], &tot);
        dbase[threadIdx.x] = e;
    }
    __syncthreads();
    const int base = blockIdx.x * RS_TILE + w * (64 * RS_ITEMS) + lane;
    u64 k[RS_ITEMS];
    u32 v[RS_ITEMS], rank[RS_ITEMS];
    const u64 lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = base + r * 64;
        const bool ok = i < n;
        k[r] = ok ? kin[i] : 0ull;
        v[r] = ok ? vin[i] : 0u;
        const u32 dg = (u32)(k[r] >> shift) & 255u;
        u64 peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const u64 bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const u32 before = ok ? wcnt[w][dg] : 0u;
        rank[r] = before + (u32)__popcll(peers & lt);
        const bool leader = ok && ((peers & lt) == 0ull);
        __builtin_amdgcn_wave_barrier();  // every lane has read its count before a leader updates it
        if (leader) wcnt[w][dg] = before + (u32)__popcll(peers);
    }
    __syncthreads();
    {   // per digit: local offsets of the tile's sorted order, per-wave offsets, global base
        const int dg = threadIdx.x;
        const u32 c0 = wcnt[0][dg], c1 = wcnt[1][dg], c2 = wcnt[2][dg], c3 = wcnt[3][dg];
        u32 tot;
        const u32 lo = block_excl_scan<u32>(c0 + c1 + c2 + c3, &tot);
        loff[dg] = lo;
        gbase[dg] = dbase[dg] + offs[dg * nb + blockIdx.x];
        woff[0][dg] = lo;
        woff[1][dg] = lo + c0;
        woff[2][dg] = lo + c0 + c1;
        woff[3][dg] = lo + c0 + c1 + c2;
    }
    __syncthreads();
    // keys into LDS in the tile's sorted order, then written out from there so that
    // consecutive lanes write consecutive addresses of a digit's run
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        if (base + r * 64 < n) {
            const u32 dg = (u32)(k[r] >> shift) & 255u;
            const u32 pl = woff[w][dg] + rank[r];
            sk[pl] = k[r];
            sv[pl] = v[r];
        }
    }
    __syncthreads();
    const int t0 = blockIdx.x * RS_TILE;
    const int tn = n - t0 < RS_TILE ? n - t0 : RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int j = threadIdx.x + r * RS_THREADS;
        if (j < tn) {
            const u64 kk = sk[j];
            const u32 dg = (u32)(kk >> shift) & 255u;
            const u32 pos = gbase[dg] + ((u32)j - loff[dg]);
            kout[pos] = kk;
            vout[pos] = sv[j];
        }
    }
}

// Per-digit exclusive scan of the per-block counts: one workgroup per digit scans that
// digit's contiguous row (digit-major table) and records the digit total.
__global__ void __launch_bounds__(SC_THREADS) k_rs_digit_scan(u32* hist, int nb, u32* digit_tot) {
    u32* h = hist + (size_t)blockIdx.x * nb;
    u32 carry = 0;
    for (int b0 = 0; b0 < nb; b0 += SC_TILE) {
        u32 v[SC_ITEMS];
        u32 s = 0;
#pragma unroll
        for (int k = 0; k < SC_ITEMS; ++k) {
            const int i = b0 + threadIdx.x * SC_ITEMS + k;
            v[k] = i < nb ? h[i] : 0u;
            s += v[k];
        }
        u32 tot;
        u32 e = block_excl_scan<u32>(s, &tot) + carry;
#pragma unroll
        for (int k = 0; k < SC_ITEMS; ++k) {
            const int i = b0 + threadIdx.x * SC_ITEMS + k;
            if (i < nb) h[i] = e;
            e += v[k];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// Sorts (key_a, val_a) in place (ping-pong through key_b / val_b; 8 passes end in _a).
void radix_sort(hipStream_t s, const DevPtrs& d, int n) {
    if (n <= 1) return;
    const int nb = (n + RS_TILE - 1) / RS_TILE;
    u64 *ki = d.key_a, *ko = d.key_b;
    u32 *vi = d.val_a, *vo = d.val_b;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, s, ki, n, shift, d.rs_hist, nb);
        hipLaunchKernelGGL(k_rs_digit_scan, dim3(256), dim3(SC_THREADS), 0, s, d.rs_hist, nb, d.rs_dtot);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, s, ki, vi, ko, vo, n, shift, d.rs_hist, nb,
                           d.rs_dtot);
        u64* tk = ki; ki = ko; ko = tk;
        u32* tv = vi; vi = vo; vo = tv;
    }
}

// ---------------------------------------------------------------------------------------
// caller-order input -> key-ordered snapshot
__global__ void __launch_bounds__(256) k_gather_input(int n, const u32* __restrict__ perm,
                                                       const double* __restrict__ x, const double* __restrict__ y,
                                                       const double* __restrict__ z, const double* __restrict__ vx,
                                                       const double* __restrict__ vy, const double* __restrict__ vz,
                                                       const double* __restrict__ m, const double* __restrict__ h,
                                                       const double* __restrict__ u, DevPtrs d, int64_t* order_out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 i = perm[q];
    const double px = x[i], py = y[i], pz = z[i], ph = h[i], pm = m[i];
    const double wx = vx[i], wy = vy[i], wz = vz[i], pu = u[i];
    d.id[q] = i;
    d.x[q] = px; d.y[q] = py; d.z[q] = pz;
    d.vx[q] = wx; d.vy[q] = wy; d.vz[q] = wz;
    d.m[q] = pm; d.h[q] = ph; d.u[q] = pu;
    d.pos4[q] = make_double4(px, py, pz, ph);
    d.vel4[q] = make_double4(wx, wy, wz, pm);
    if (order_out) order_out[q] = (int64_t)i;
}

void launch_gather_input(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* x, const double* y,
                         const double* z, const double* vx, const double* vy, const double* vz, const double* m,
                         const double* h, const double* u, int64_t* order_out) {
    if (dm.n > 0)
        hipLaunchKernelGGL(k_gather_input, dim3((dm.n + 255) / 256), dim3(256), 0, s, dm.n, d.val_a, x, y, z, vx,
                           vy, vz, m, h, u, d, order_out);
}
