// Neighbour search (Sec. 2.1 of arXiv:2007.03097, last paragraph: the traversal runs for
// a group of particles, prunes with the node bounds and builds one neighbour list per
// particle).
//
// One wavefront per target group (at most group_size consecutive particles of one compact
// octree cell), in an XCD-aware loop over the groups (one group per workgroup at the
// default grid, which holds a workgroup per expected group).
//  1. Group box and largest h by wave reductions.
//  2. Wide tree walk: up to 64 nodes are tested at once, one per lane, against the group
//     box.  A node survives when the squared gap between the boxes, summed in the same
//     operation order as the pair test, is below (hmax_group + hmax_node)^2; rounding is
//     monotone in every operation, so no true neighbour pair is ever pruned.  Surviving
//     leaves go to a candidate list, surviving internal nodes push their children.  The
//     candidate list is matched (step 3) whenever it fills, so any number of candidates
//     is handled with fixed LDS.
//  3. Each candidate particle is tested against the group box (conservatively, as the
//     nodes are); survivors are staged in an LDS ring and matched 64 at a time: lane
//     (tp, phi) tests the block of sources phi*T .. phi*T + T - 1 (T = group_size/2) against
//     its two targets tp and tp + T with the exact predicate
//     fl(fl(fl(dx dx) + fl(dy dy)) + fl(dz dz)) < fl(t t), recording hits as bits (two
//     targets per lane halve the LDS reads per pair test).  The predicate is screened in FP32
//     (fp32_screen below): the screen decides every pair outside a proven error margin, the
//     few pairs inside it take the FP64 expression, so the lists are those of the FP64
//     predicate bit for bit.  The OR of all lanes' bits is the tile's part of the group's
//     source union U (sources that are a neighbour of at least one target), appended to
//     U in staging order.  The 64/T lanes of a target then take consecutive slot ranges
//     and write, for each hit, the source's index in U.
// Outputs per group (n_g targets starting at sorted position s):
//   uni[s*cap + i], i < ucnt[group]: particle index of the i-th member of U;
//   nbr[s*cap + k*n_g + t]: slot k of target t, a 16-bit index into U (|U| <= UNION_MAX),
//   ascending in k; the blocks of all groups tile exactly n * cap entries, and consumers
//   reading slot k of consecutive targets read consecutive entries.
// The pair kernels stage U in LDS and read their sources there.
#include "common.h"

constexpr int WALK_STACK = 512;
constexpr int WALK_CAND = 256;

constexpr int TILE_RING = 128;

// Group-level state of the matching step.
struct GroupBox {
    double lo[3], hi[3], hg;
};

// FP32 screen of the exact predicate.  Coordinates are offsets from the group origin o (the
// group's first target), each formed in FP64 and rounded to FP32; h is rounded to FP32.
// With u = 2^-24 and E the largest per-axis offset of a target from o, the screen values
//   r2' = fma(dx', dx', fma(dy', dy', dz' dz')),  t' = fl(h_a' + h_b')
// (dx' = fl(x_a' - x_b') ...) give r2' and t'^2 within 3.6u E^2 + 10.7u r^2 and 4.1u t^2 of the
// exact r^2 and t^2 = (h_a + h_b)^2 (offset errors grow with |x - o| <= E + |dx|), and the
// FP64 expressions differ from them by O(2^-53).  The screen value d' = fma(t', t', -r2')
// rounds once, so with t2' = fl(t'^2) and
//   M = 2^-21 E^2 + 2^-19 t2' + 2^-100   (about twice the bound; the last term covers FP32
//                                          underflow)
// the FP64 predicate holds when d' > M and fails when d' < -M.  Pairs with
// |d'| <= M, and any NaN or overflow, are undecided and take the FP64 expression.  FP32
// arithmetic issues at twice the FP64 rate on this GPU and the staged records halve.
struct Screen {
    double o[3];   // group origin
    float me;      // 2^-21 E^2 + 2^-100, rounded up
};

// Each lane serves two targets of the group, tp and tp + TP (TP = group_size / 2), and a
// block of B = TP staged sources; the P = 64 / TP lanes with the same tp cover the tile.
// One LDS read of a source feeds two pair tests.
template <int TP_>
struct LaneTargets {
    static constexpr int TP = TP_, P = 64 / TP_;
    float4 a, b;    // targets tp and tp + TP: FP32 offsets from the origin, h
    bool va, vb;    // they exist
    int tp, phi;
    int cnt_a, cnt_b;
};

__device__ __forceinline__ float4 offset_rec(const double4& p, const Screen& S) {
    return make_float4((float)(p.x - S.o[0]), (float)(p.y - S.o[1]), (float)(p.z - S.o[2]), (float)p.w);
}

// Margin of the screen for target a against a tile whose sources have |h| <= hm:
// M' = fma(fl(fl(|h_a| + hm)^2), 2^-19, me) is at least the margin fma(t2', 2^-19, me) of
// each of those pairs (t2' = fl(fl(h_a + h_b)^2), every operation monotone), so deciding
// with M' keeps the screen's guarantee and only leaves a few more pairs undecided.  A NaN
// h makes M' NaN and every pair of the target undecided.
__device__ __forceinline__ float tile_margin(float ha, float hm, float me) {
    const float tt = fabsf(ha) + hm;
    return fmaf(tt * tt, 0x1p-19f, me);
}

// d' = fma(t', t', -r2') of one pair (the screen value; see fp32_screen above).
__device__ __forceinline__ float screen_d(const float4& a, const float4& s) {
    const float dx = a.x - s.x, dy = a.y - s.y, dz = a.z - s.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float tt = a.w + s.w;
    return fmaf(tt, tt, -r2);
}

// Largest |h| of the tn (>= 1) sources of the tile at ring positions head .., over the wave:
// the bits of a non-negative float order as unsigned integers (a NaN above every number).
__device__ __forceinline__ float tile_hmax(const float4* tile, int head, int tn) {
    const int lane = lane_id();
    u32 v = lane < tn ? __float_as_uint(fabsf(tile[(head + lane) & (TILE_RING - 1)].w)) : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (u32)__shfl_xor((int)v, d, 64));
    return __uint_as_float(v);
}

// The exact FP64 predicate for the pairs the screen left undecided (bit i = tile source i).
__device__ void resolve_exact(u32 q, const double4& A, int head, int j0, const int* tsrc,
                              const double4* __restrict__ pos4, u32& hits) {
    while (q) {
        const int it = __ffs(q) - 1;
        q &= q - 1;
        const double4 s = pos4[tsrc[(head + j0 + it) & (TILE_RING - 1)]];
        const double dx = A.x - s.x, dy = A.y - s.y, dz = A.z - s.z;
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        const double tt = A.w + s.w;
        if (r2 < tt * tt) hits |= 1u << it;
    }
}

// Slots for one target's hits: the P lanes of the target take consecutive slot ranges in
// phi order, each in ascending source order; the entry is the source's index in the union.
template <int TP>
__device__ __forceinline__ void append_hits(u32 bits, int t, int& cnt, const LaneTargets<TP>& L, u64 ub, int ucnt,
                                            int gy, int cap, u16* mylist) {
    const int lane = lane_id();
    const int mine = __popc(bits);
    int incl = mine;
    for (int d = L.TP; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    const int tot = __shfl(incl, L.tp + L.TP * (L.P - 1), 64);
    int slot = cnt + incl - mine;
    const int j0 = L.phi * L.TP;
    while (bits) {
        const int it = __ffs(bits) - 1;
        bits &= bits - 1;
        const int j = j0 + it;
        // past UNION_MAX (an overflow the kernel reports) entries stay at the last index, in bounds
        if (slot < cap) mylist[slot * gy + t] = (u16)min(ucnt + __popcll(ub & ((1ull << j) - 1ull)), UNION_MAX - 1);
        ++slot;
    }
    cnt += tot;
}

// Exact predicate fl(fl(fl(dx dx) + fl(dy dy)) + fl(dz dz)) < fl(t t), t = fl(h_a + h_b),
// for the 64 (or, at the end, fewer) filtered sources at ring positions head .. head+tn-1
// (FP32 screen, FP64 for the undecided pairs); hits go to the group's union and to the
// targets' lists.
template <int TP>
__device__ __forceinline__ void test_tile(int head, int tn, const float4* tile, const int* tsrc, LaneTargets<TP>& L,
                                          float me, const double4* __restrict__ pos4, int gx, int gy, int cap,
                                          u16* mylist, int* myuni, int ulim, int& ucnt) {
    const int lane = lane_id();
    const int j0 = L.phi * TP;
    const int je = min(max(tn - j0, 0), TP);  // sources of this lane's block
    const u32 valid = je >= 32 ? 0xffffffffu : (1u << je) - 1u;
    const float hm = tile_hmax(tile, head, tn);
    const float Ma = tile_margin(L.a.w, hm, me), Mb = tile_margin(L.b.w, hm, me);
    // head is a multiple of 64, so the block's TP ring entries are contiguous; entries past
    // the block's end are stale records whose bits are masked off below
    const float4* blk = tile + ((head + j0) & (TILE_RING - 1));
    u32 ba = 0, bb = 0;
    u64 und = 0;  // lanes with an undecided pair
    // sources in descending order, each decision shifted in at bit 0, so that bit it ends up
    // holding source it; one ballot per comparison keeps the undecided masks in scalar registers
#pragma unroll 4
    for (int it = TP - 1; it >= 0; --it) {
        const float4 s = blk[it];
        const float da = screen_d(L.a, s), db = screen_d(L.b, s);
        ba = ba + ba + (da > Ma ? 1u : 0u);
        bb = bb + bb + (db > Mb ? 1u : 0u);
        und |= __builtin_amdgcn_ballot_w64(!(fabsf(da) > Ma)) | __builtin_amdgcn_ballot_w64(!(fabsf(db) > Mb));
    }
    ba &= L.va ? valid : 0u;
    bb &= L.vb ? valid : 0u;
    if (und) {  // rare: the lanes concerned redo their block's undecided pairs in FP64
        u32 qa = 0, qb = 0;
        if ((und >> lane) & 1ull) {
            for (int it = 0; it < je; ++it) {
                const float4 s = blk[it];
                if (!(fabsf(screen_d(L.a, s)) > Ma)) qa |= 1u << it;
                if (!(fabsf(screen_d(L.b, s)) > Mb)) qb |= 1u << it;
            }
            if (!L.va) qa = 0u;
            if (!L.vb) qb = 0u;
        }
        if (qa) resolve_exact(qa, pos4[gx + L.tp], head, j0, tsrc, pos4, ba);
        if (qb) resolve_exact(qb, pos4[gx + L.tp + TP], head, j0, tsrc, pos4, bb);
    }
    // union of the tile, bit j = ring entry head + j
    u64 ub = (u64)(ba | bb) << j0;
    for (int d = 1; d < 64; d <<= 1) ub |= __shfl_xor(ub, d, 64);
    if ((ub >> lane) & 1ull) {
        const int r = ucnt + __popcll(ub & lanemask_lt());
        if (r < ulim) myuni[r] = tsrc[(head + lane) & (TILE_RING - 1)];
    }
    append_hits(ba, L.tp, L.cnt_a, L, ub, ucnt, gy, cap, mylist);
    append_hits(bb, L.tp + L.TP, L.cnt_b, L, ub, ucnt, gy, cap, mylist);
    ucnt += __popcll(ub);
}

// Matching of the group's targets against the particles of the nc candidate leaves in
// cand[] (node ids; reused for the leaves' first particles).  Each candidate particle is
// first tested against the group box, in the same monotone operation order as the node
// test (gap^2 < (hmax_group + h_b)^2), so no true neighbour is dropped; survivors enter an
// LDS ring and are matched 64 at a time.  Sources left in the ring (< 64) are matched by
// the caller's final flush.
template <int TP>
__device__ void match_candidates(int nc, int* cand, int* coff, float4* tile, int* tsrc, int& head, int& tail,
                                 const GroupBox& gb, const Screen& S, const int4* __restrict__ topo,
                                 const double4* __restrict__ pos4, LaneTargets<TP>& L, int gx, int gy, int cap,
                                 u16* mylist, int* myuni, int ulim, int& ucnt) {
    const int lane = lane_id();
    const u64 lt = lanemask_lt();
    int carry = 0;
    for (int j0 = 0; j0 < nc; j0 += 64) {
        const int j = j0 + lane;
        int c = 0, st = 0;
        if (j < nc) {
            const int4 tp = topo[cand[j]];
            st = tp.x;
            c = tp.y;
        }
        const int incl = wave_incl_scan(c);
        __syncthreads();
        if (j < nc) {
            cand[j] = st;
            coff[j] = carry + incl - c;
        }
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) coff[nc] = carry;
    __syncthreads();
    const int total = carry;
    for (int p0 = 0; p0 < total; p0 += 64) {
        const int p = p0 + lane;
        bool pass = false;
        int src = 0;
        double4 b = make_double4(0, 0, 0, 0);
        if (p < total) {
            int a = 0, bb = nc - 1;
            while (a < bb) {  // largest j with coff[j] <= p
                const int mid = (a + bb + 1) >> 1;
                if (coff[mid] <= p) a = mid;
                else bb = mid - 1;
            }
            src = cand[a] + (p - coff[a]);
            b = pos4[src];
            const double gx = fmax(0.0, fmax(b.x - gb.hi[0], gb.lo[0] - b.x));
            const double gy2 = fmax(0.0, fmax(b.y - gb.hi[1], gb.lo[1] - b.y));
            const double gz = fmax(0.0, fmax(b.z - gb.hi[2], gb.lo[2] - b.z));
            double r2 = gx * gx + gy2 * gy2;
            r2 = r2 + gz * gz;
            const double tt = gb.hg + b.w;
            pass = r2 < tt * tt;
        }
        const u64 bal = __ballot(pass);
        if (pass) {
            const int r = (tail + __popcll(bal & lt)) & (TILE_RING - 1);
            tile[r] = offset_rec(b, S);
            tsrc[r] = src;
        }
        tail += __popcll(bal);
        __syncthreads();
        if (tail - head >= 64) {
            test_tile(head, 64, tile, tsrc, L, S.me, pos4, gx, gy, cap, mylist, myuni, ulim, ucnt);
            head += 64;
        }
        __syncthreads();
    }
}

// 96 VGPRs (five waves per SIMD, no spills) against 110 (four) unconstrained: the walk's
// dependent loads need the extra wave more than the screen needs the registers.
template <int TP>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) k_nbr_lists(DevCtl* ctl, const int4* __restrict__ group, int gsz, int cap,
                                                  const int4* __restrict__ topo, const double4* __restrict__ nbox_lo,
                                                  const double4* __restrict__ nbox_hi, const double4* __restrict__ pos4,
                                                  u16* __restrict__ nbr, int* __restrict__ nbr_cnt,
                                                  int* __restrict__ list_base, int* __restrict__ uni,
                                                  int* __restrict__ ucnt_out) {
    __shared__ int stack[WALK_STACK];
    __shared__ int cand[WALK_CAND];
    __shared__ int coff[WALK_CAND + 1];
    __shared__ float4 tile[TILE_RING];
    __shared__ int tsrc[TILE_RING];
    const int lane = lane_id();
    const u64 lt = lanemask_lt();
    LaneTargets<TP> L;
    L.tp = lane & (L.TP - 1);
    L.phi = lane / L.TP;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
        const int4 g = group[gi];
        L.va = L.tp < g.y;
        L.vb = L.tp + L.TP < g.y;
        const double4 A = L.va ? pos4[g.x + L.tp] : make_double4(0, 0, 0, 0);
        const double4 B = L.vb ? pos4[g.x + L.tp + L.TP] : make_double4(0, 0, 0, 0);
        L.cnt_a = L.cnt_b = 0;
        GroupBox gb;
        gb.lo[0] = wave_min(fmin(L.va ? A.x : INFINITY, L.vb ? B.x : INFINITY));
        gb.lo[1] = wave_min(fmin(L.va ? A.y : INFINITY, L.vb ? B.y : INFINITY));
        gb.lo[2] = wave_min(fmin(L.va ? A.z : INFINITY, L.vb ? B.z : INFINITY));
        gb.hi[0] = wave_max(fmax(L.va ? A.x : -INFINITY, L.vb ? B.x : -INFINITY));
        gb.hi[1] = wave_max(fmax(L.va ? A.y : -INFINITY, L.vb ? B.y : -INFINITY));
        gb.hi[2] = wave_max(fmax(L.va ? A.z : -INFINITY, L.vb ? B.z : -INFINITY));
        gb.hg = wave_max(fmax(L.va ? A.w : 0.0, L.vb ? B.w : 0.0));
        Screen S;
        {
            const double4 o = pos4[g.x];
            S.o[0] = o.x;
            S.o[1] = o.y;
            S.o[2] = o.z;
            double E = 0.0;
            for (int c = 0; c < 3; ++c) E = fmax(E, fmax(gb.hi[c] - S.o[c], S.o[c] - gb.lo[c]));
            S.me = (float)((ldexp(E * E, -21) + 0x1p-100) * (1.0 + 0x1p-20));  // rounded up
        }
        L.a = offset_rec(A, S);
        L.b = offset_rec(B, S);
        const double* lo = gb.lo;
        const double* hi = gb.hi;
        const double hg = gb.hg;
        u16* mylist = nbr + (size_t)g.x * (size_t)cap;
        int* myuni = uni + (size_t)g.x * (size_t)cap;
        const int ulim = min(g.y * cap, UNION_MAX);
        int ucnt = 0, head = 0, tail = 0;
        const int root = g.z < 0 ? 0 : ctl->level_off[3] + g.z;
        __syncthreads();
        if (lane == 0) stack[0] = root;
        int sp = 1, nc = 0, iters = 0;
        bool overflow = false;
        __syncthreads();
        while (sp > 0) {
            if (++iters > (1 << 20)) {  // bounded: every wave leaves the loop
                overflow = true;
                break;
            }
            if (nc + 64 > WALK_CAND) {
                match_candidates(nc, cand, coff, tile, tsrc, head, tail, gb, S, topo, pos4, L, g.x, g.y, cap, mylist,
                                 myuni, ulim, ucnt);
                nc = 0;
            }
            // pop at most as many nodes as the free stack can take the children of (8 each)
            int k = sp < 64 ? sp : 64;
            const int room = (WALK_STACK - sp) / 8;
            if (k > room) k = room > 1 ? room : 1;
            const int node = lane < k ? stack[sp - k + lane] : -1;
            __syncthreads();
            sp -= k;
            bool hit = false;
            int4 tp = make_int4(0, 0, 0, 0);
            if (node >= 0) {
                tp = topo[node];
                const double4 a = nbox_lo[node], b = nbox_hi[node];
                const double gx = fmax(0.0, fmax(a.x - hi[0], lo[0] - b.x));
                const double gy = fmax(0.0, fmax(a.y - hi[1], lo[1] - b.y));
                const double gz = fmax(0.0, fmax(a.z - hi[2], lo[2] - b.z));
                double r2 = gx * gx + gy * gy;
                r2 = r2 + gz * gz;
                const double tt = hg + a.w;
                hit = r2 < tt * tt;
            }
            const bool isleaf = hit && tp.w;
            const u64 bl = __ballot(isleaf);
            if (isleaf) cand[nc + __popcll(bl & lt)] = node;
            nc += __popcll(bl);
            const int nch = (hit && !tp.w) ? tp.y : 0;
            const int incl = wave_incl_scan(nch);
            const int tot = __shfl(incl, 63, 64);
            if (sp + tot > WALK_STACK) {
                overflow = true;
                break;
            }
            for (int j = 0; j < nch; ++j) stack[sp + incl - nch + j] = tp.x + j;
            sp += tot;
            __syncthreads();
        }
        __syncthreads();
        if (!overflow) {
            match_candidates(nc, cand, coff, tile, tsrc, head, tail, gb, S, topo, pos4, L, g.x, g.y, cap, mylist,
                             myuni, ulim, ucnt);
            if (tail > head)
                test_tile(head, tail - head, tile, tsrc, L, S.me, pos4, g.x, g.y, cap, mylist, myuni, ulim, ucnt);
            __syncthreads();
        } else if (lane == 0)
            set_err(ctl, ERR_WALK_STACK);
        if (lane == 0) {
            ucnt_out[gi] = overflow ? 0 : (ucnt < ulim ? ucnt : ulim);
            if (ucnt > UNION_MAX) set_err(ctl, ERR_UNION_CAP);
        }
        if (L.phi == 0) {
            for (int s = 0; s < 2; ++s) {
                if (!(s ? L.vb : L.va)) continue;
                const int q = g.x + L.tp + s * L.TP;
                const int cnt = s ? L.cnt_b : L.cnt_a;
                nbr_cnt[q] = overflow ? 0 : (cnt < cap ? cnt : cap);
                list_base[q] = overflow ? -1 : gi;
                if (cnt > cap) {
                    set_err(ctl, ERR_NBR_CAP);
                    atomicMax(&ctl->nbr_max, cnt);
                }
            }
        }
    }
}

void launch_nbr_lists(hipStream_t s, const DevPtrs& d, const Dims& dm) {
    if (dm.n <= 0) return;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size, dm.nbr_cap,
                           d.topo, d.nbox_lo, d.nbox_hi, d.pos4, d.nbr, d.nbr_cnt, d.nbr_base, d.uni, d.ucnt);
    };
    switch (dm.group_size) {  // validated at context creation: 8, 16, 32 or 64
        case 8: go(k_nbr_lists<4>); break;
        case 16: go(k_nbr_lists<8>); break;
        case 32: go(k_nbr_lists<16>); break;
        default: go(k_nbr_lists<32>); break;
    }
}

// ---- CSR export in caller order (test and inspection path)
__global__ void k_csr_count(int n, const u32* __restrict__ id, const int* __restrict__ cnt, int64_t* counts) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) counts[id[q]] = cnt[q];
}

void launch_csr_count(hipStream_t s, const DevPtrs& d, const Dims& dm, int64_t* counts_caller) {
    if (dm.n > 0) hipLaunchKernelGGL(k_csr_count, dim3((dm.n + 255) / 256), dim3(256), 0, s, dm.n, d.id, d.nbr_cnt,
                                     counts_caller);
}

__global__ void k_csr_fill(int n, int gsz, int cap, const int4* __restrict__ group, const u32* __restrict__ id,
                           const int* __restrict__ cnt, const int* __restrict__ gidx, const u16* __restrict__ nbr,
                           const int* __restrict__ uni, const int64_t* __restrict__ off, int32_t* idx) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int c = cnt[q], g = gidx[q];
    if (g < 0) return;
    const int4 gr = group[g];
    const u16* lst = nbr + (size_t)gr.x * cap + (q - gr.x);
    const int* un = uni + (size_t)gr.x * cap;
    int32_t* out = idx + off[id[q]];
    for (int k = 0; k < c; ++k) {   // insertion sort by caller index while copying
        const int32_t v = (int32_t)id[un[lst[k * gr.y]]];
        int j = k;
        while (j > 0 && out[j - 1] > v) {
            out[j] = out[j - 1];
            --j;
        }
        out[j] = v;
    }
}

void launch_csr_fill(hipStream_t s, const DevPtrs& d, const Dims& dm, const int64_t* offsets, int32_t* idx) {
    if (dm.n > 0) hipLaunchKernelGGL(k_csr_fill, dim3((dm.n + 255) / 256), dim3(256), 0, s, dm.n, dm.group_size,
                                     dm.nbr_cap, d.group, d.id, d.nbr_cnt, d.nbr_base, d.nbr, d.uni, offsets, idx);
}
