// Octree over sorted keys (Sec. 2.1 "Tree topology" of arXiv:2007.03097, Fig. 1).
//
// A cell at level l is the run of sorted particles sharing the first l 3-bit digits of
// their keys.  The root (level 0) is a node; a cell is a node when its parent cell is a
// node holding more than leaf_size particles (and l <= 21); a node is a leaf when it holds
// at most leaf_size particles, or at level 21.  This is the paper's refine-until-isolated
// rule with "isolated" widened to leaf_size particles.
//
// Data-parallel construction, no recursion:
//   lcp[i]   = leading equal digits of keys i-1 and i (-1 at i = 0 and i = n): cell
//              boundaries at level l are the positions with lcp < l.
//   lvl[i]   = level of the leaf holding i = 1 + min{v : the nearest boundaries with
//              lcp <= v on both sides of i are at most leaf_size apart}, found in one
//              pass over a window of lcp values in LDS (see window_level).
//   position i starts the nodes of levels lcp[i]+1 .. lvl[i]; an exclusive scan of those
//   counts numbers the nodes in pre-order.  A stable counting sort by level turns that
//   into breadth-first order, where the children of a node are a contiguous run of the
//   next level.  Moments are aggregated bottom-up one level at a time.
//   The largest nodes holding at most 4 * group_size particles form compact "group cells";
//   each is split into target groups of at most group_size consecutive particles, so a
//   group never spans two distant cells of the space-filling curve.
#include "common.h"

constexpr int TB = 256;          // positions per block in the leaf-level kernel
constexpr int MAX_WIN = 64;      // largest supported leaf_size

// Level of the smallest cell around position ci that holds at most win particles:
// 1 + min{v : the nearest boundaries with lcp <= v on both sides are at most win apart}.
// With ML(t) = min c[ci-t .. ci] and MR(k) = min c[ci+1 .. ci+k], a level v qualifies
// exactly when ML(t) <= v and MR(k) <= v for some t < win, k >= 1, t + k <= win; both
// minima only fall as t, k grow, so the smallest v is min over t of max(ML(t), MR(win - t)).
// One branch-free pass; this thread's MR(k) sits at mr[(k - 1) * TB] in LDS (threads of a
// wave write neighbouring bytes).
__device__ __forceinline__ int window_level(const signed char* c, int ci, int win, signed char* mr) {
    int m = 127;
    for (int k = 1; k <= win; ++k) {
        const int v = c[ci + k];
        m = v < m ? v : m;
        mr[(k - 1) * TB] = (signed char)m;
    }
    int best = 127, ml = 127;
    for (int t = 0; t < win; ++t) {
        const int v = c[ci - t];
        ml = v < ml ? v : ml;
        const int r = mr[(win - 1 - t) * TB];
        const int x = ml > r ? ml : r;
        best = x < best ? x : best;
    }
    const int L = best + 1;
    return L > MAX_LEVEL ? MAX_LEVEL : L;
}

// window_level with the leaf capacity W known at compile time: the running minima MR(k) stay
// in registers (the same values, the same pairing of ML(t) with MR(W - t)).
template <int W>
__device__ __forceinline__ int window_level_w(const signed char* c, int ci) {
    int mr[W];
    int m = 127;
#pragma unroll
    for (int k = 1; k <= W; ++k) {
        const int v = c[ci + k];
        m = v < m ? v : m;
        mr[k - 1] = m;
    }
    int best = 127, ml = 127;
#pragma unroll
    for (int t = 0; t < W; ++t) {
        const int v = c[ci - t];
        ml = v < ml ? v : ml;
        const int r = mr[W - 1 - t];
        const int x = ml > r ? ml : r;
        best = x < best ? x : best;
    }
    const int L = best + 1;
    return L > MAX_LEVEL ? MAX_LEVEL : L;
}

// Per sorted position: lcp, leaf level (leaf capacity win) and the node / leaf-start counts
// for the pre-order scan.  Also clears the per-level node counters (block 0) and the
// group-cell flags of every position, which later kernels of the build fill in.  W > 0: the
// leaf capacity is W (= win) and the window runs in registers; W = 0: any win, through LDS.
template <int W>
__global__ void __launch_bounds__(TB) k_leaf_levels(const u64* __restrict__ key, int n, int win, int min_level,
                                                    signed char* lcp, unsigned char* lvl, u64* scan_in, DevCtl* ctl,
                                                    u32* gflag) {
    if (blockIdx.x == 0 && threadIdx.x < 24) ctl->level_count[threadIdx.x] = 0;
    __shared__ signed char c[TB + 2 * MAX_WIN + 2];
    __shared__ signed char mrow[W > 0 ? 1 : TB * MAX_WIN];
    const int b0 = blockIdx.x * TB;
    const int lo = b0 - win;                      // c[j] holds position lo + j
    const int cnt = TB + 2 * win + 1;
    for (int j = threadIdx.x; j < cnt; j += TB) {
        const int p = lo + j;
        int v = -1;
        if (p > 0 && p < n) v = lcp_digits(key[p - 1], key[p]);
        c[j] = (signed char)v;
    }
    __syncthreads();
    const int i = b0 + threadIdx.x;
    if (i >= n) return;
    const int ci = i - lo;
    int L;
    if constexpr (W > 0) L = window_level_w<W>(c, ci);
    else L = window_level(c, ci, win, mrow + threadIdx.x);
    if (L < min_level) L = min_level;
    const int cc = c[ci];
    const int nodes = L > cc ? L - cc : 0;
    lcp[i] = (signed char)cc;
    lvl[i] = (unsigned char)L;
    scan_in[i] = ((u64)nodes << 32) | (u64)(nodes > 0 ? 1u : 0u);
    gflag[i] = 0u;
    if (i == n - 1) {
        lcp[n] = -1;
        gflag[n] = 0u;
    }
}

// Group cells: the largest nodes holding at most gcap particles (at or below min_level),
// plus leaves that hold more (runs of equal keys).  They partition the sorted particles.
// Each is cut into target groups of at most gsz consecutive particles: the first position
// of every group is flagged and the group's size recorded there.
__global__ void k_group_starts(const DevCtl* __restrict__ ctl, int gcap, int gsz, int min_level,
                               const int4* __restrict__ topo, const int* __restrict__ parent,
                               const int2* __restrict__ range, u32* gflag, u32* gsize) {
    const int nn = ctl->n_nodes;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nn; b += gridDim.x * blockDim.x) {
        const int4 tp = topo[b];
        const bool fits = range[b].y <= gcap && tp.z >= min_level;
        if (!(fits || tp.w)) continue;
        const int p = parent[b];
        bool pfits = false;
        if (p >= 0) pfits = range[p].y <= gcap && topo[p].z >= min_level;
        if (pfits) continue;
        const int2 r = range[b];
        const int e = r.x + r.y;
        for (int k = r.x; k < e; k += gsz) {
            gflag[k] = 1u;
            gsize[k] = (u32)min(gsz, e - k);
        }
    }
}

// Target groups in sorted order: group gscan[i] starts at each flagged position i.
__global__ void k_emit_groups(int n, int batched, DevCtl* ctl, const u32* __restrict__ gflag,
                              const u32* __restrict__ gscan, const u32* __restrict__ gsize,
                              const u64* __restrict__ key, const int* __restrict__ seg_root_rank, int4* group) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ctl->n_groups = (int)gscan[n];
    if (i < n && gflag[i]) {
        const int rank = batched ? seg_root_rank[(int)((key[i] >> 54) & 511ull)] : -1;
        group[gscan[i]] = make_int4(i, (int)gsize[i], rank, 0);
    }
}

// Pre-order node records, leaf table and per-level node counts.  A grid-stride loop over
// positions; the level counts are wave-aggregated into LDS and added to the global counts
// once per workgroup, so the 24 global counters see few atomics.
__global__ void __launch_bounds__(256) k_emit_nodes(int n, const signed char* __restrict__ lcp,
                                                     const unsigned char* __restrict__ lvl,
                                                     const u64* __restrict__ scan, unsigned char* pre_level,
                                                     unsigned char* pre_leaf, int* pre_start, int* leaf_start,
                                                     int* leaf_pre, DevCtl* ctl, int node_cap) {
    __shared__ int hist[24];
    if (threadIdx.x < 24) hist[threadIdx.x] = 0;
    __syncthreads();
    const u64 tot = scan[n];
    const int n_nodes = (int)(tot >> 32), n_leaves = (int)(tot & 0xffffffffu);
    const int stride = gridDim.x * blockDim.x;
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
        const int i = i0 + threadIdx.x;
        int c = MAX_LEVEL, L = -1;
        if (i < n) {
            c = lcp[i];
            L = lvl[i];
        }
        if (L > c) {
            const u64 sv = scan[i];
            const int base = (int)(sv >> 32), lf = (int)(sv & 0xffffffffu);
            for (int l = c + 1; l <= L; ++l) {
                const int idx = base + (l - c - 1);
                if (idx < node_cap) {
                    pre_level[idx] = (unsigned char)l;
                    pre_leaf[idx] = (unsigned char)(l == L);
                    pre_start[idx] = i;
                }
            }
            leaf_start[lf] = i;
            leaf_pre[lf] = base + (L - c - 1);
        }
        // nodes per level: position i starts one node at each level c+1 .. L
        const u64 any = __ballot(L > c);
        if (any) {
            for (int l = 0; l <= MAX_LEVEL; ++l) {
                const int k = __popcll(__ballot(c < l && l <= L));
                if (k && lane_id() == 0) atomicAdd(&hist[l], k);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->n_nodes = n_nodes < node_cap ? n_nodes : node_cap;
        ctl->n_leaves = n_leaves;
        leaf_start[n_leaves] = n;
        if (n_nodes > node_cap) set_err(ctl, ERR_NODE_CAP);
    }
    __syncthreads();
    if (threadIdx.x < 24 && hist[threadIdx.x]) atomicAdd(&ctl->level_count[threadIdx.x], hist[threadIdx.x]);
}


// Stable counting sort of pre-order nodes by level (2048-node tiles, 5-bit digit).
constexpr int LS_THREADS = 256, LS_ITEMS = 8, LS_TILE = LS_THREADS * LS_ITEMS, LS_WAVES = LS_THREADS / 64;

__global__ void __launch_bounds__(LS_THREADS) k_lsort_hist(const DevCtl* __restrict__ ctl,
                                                          const unsigned char* __restrict__ pre_level, int* hist) {
    __shared__ int h[24];
    const int nn = ctl->n_nodes;
    const int ntiles = (nn + LS_TILE - 1) / LS_TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        if (threadIdx.x < 24) h[threadIdx.x] = 0;
        __syncthreads();
        for (int r = 0; r < LS_ITEMS; ++r) {
            const int i = tile * LS_TILE + r * LS_THREADS + threadIdx.x;
            if (i < nn) atomicAdd(&h[pre_level[i]], 1);
        }
        __syncthreads();
        if (threadIdx.x < 24) hist[tile * 24 + threadIdx.x] = h[threadIdx.x];
        __syncthreads();
    }
}

// One wave per level (24): the level's first breadth-first index (level_off, the prefix of
// the level counts; written here for every later kernel), then the exclusive scan of that
// level's tile counts offset by it.
__global__ void __launch_bounds__(64) k_lsort_scan(DevCtl* ctl, int* hist) {
    const int l = blockIdx.x;
    const int nn = ctl->n_nodes;
    const int ntiles = (nn + LS_TILE - 1) / LS_TILE;
    int carry = 0;
    for (int k = 0; k < l; ++k) carry += ctl->level_count[k];
    if (lane_id() == 0) ctl->level_off[l] = carry;
    for (int t0 = 0; t0 < ntiles; t0 += 64) {
        const int t = t0 + lane_id();
        const int v = t < ntiles ? hist[t * 24 + l] : 0;
        const int inc = wave_incl_scan(v);
        if (t < ntiles) hist[t * 24 + l] = carry + inc - v;
        carry += __shfl(inc, 63, 64);
    }
}

__global__ void __launch_bounds__(LS_THREADS) k_lsort_scatter(const DevCtl* __restrict__ ctl,
                                                             const unsigned char* __restrict__ pre_level,
                                                             const int* __restrict__ hist, int* pre_to_bfs,
                                                             int* bfs_to_pre) {
    __shared__ int wcnt[LS_WAVES][24];
    __shared__ int woff[LS_WAVES][24];
    const int nn = ctl->n_nodes;
    const int ntiles = (nn + LS_TILE - 1) / LS_TILE;
    const int w = threadIdx.x >> 6, lane = lane_id();
    const u64 lt = lanemask_lt();
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int j = threadIdx.x; j < LS_WAVES * 24; j += LS_THREADS) (&wcnt[0][0])[j] = 0;
        __syncthreads();
        const int base = tile * LS_TILE + w * (64 * LS_ITEMS) + lane;
        int rank[LS_ITEMS], lev[LS_ITEMS];
        for (int r = 0; r < LS_ITEMS; ++r) {
            const int i = base + r * 64;
            const bool ok = i < nn;
            const int dg = ok ? pre_level[i] : 0;
            lev[r] = dg;
            u64 peers = __ballot(ok);
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                const bool bit = (dg >> b) & 1;
                const u64 bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const int before = ok ? wcnt[w][dg] : 0;
            rank[r] = before + __popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();  // every lane has read its count before a leader updates it
            if (ok && (peers & lt) == 0ull) wcnt[w][dg] = before + __popcll(peers);
        }
        __syncthreads();
        if (threadIdx.x < 24) {
            int acc = hist[tile * 24 + threadIdx.x];
            for (int q = 0; q < LS_WAVES; ++q) {
                woff[q][threadIdx.x] = acc;
                acc += wcnt[q][threadIdx.x];
            }
        }
        __syncthreads();
        for (int r = 0; r < LS_ITEMS; ++r) {
            const int i = base + r * 64;
            if (i < nn) {
                const int bfs = woff[w][lev[r]] + rank[r];
                pre_to_bfs[i] = bfs;
                bfs_to_pre[bfs] = i;
            }
        }
        __syncthreads();
    }
}

// Topology in breadth-first order: leaf -> particle range; internal -> children range.
__global__ void __launch_bounds__(256) k_finalize(DevCtl* ctl, const unsigned char* __restrict__ pre_level,
                                                   const unsigned char* __restrict__ pre_leaf,
                                                   const int* __restrict__ pre_start, const int* __restrict__ pre_to_bfs,
                                                   const int* __restrict__ bfs_to_pre, const signed char* __restrict__ lcp,
                                                   const u64* __restrict__ scan, const int* __restrict__ leaf_start,
                                                   int4* topo, int* parent, int* counter, int2* range) {
    const int nn = ctl->n_nodes;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nn; b += gridDim.x * blockDim.x) {
        const int pre = bfs_to_pre[b];
        const int l = pre_level[pre], s = pre_start[pre];
        counter[b] = 0;
        if (b == 0) parent[0] = -1;
        if (pre_leaf[pre]) {
            const int lf = (int)(scan[s] & 0xffffffffu);
            const int cnt = leaf_start[lf + 1] - s;
            topo[b] = make_int4(s, cnt, l, 1);
            range[b] = make_int2(s, cnt);
        } else if (pre + 1 >= nn) {  // only with a truncated (over-capacity) tree
            topo[b] = make_int4(s, 0, l, 1);
            range[b] = make_int2(s, 0);
        } else {
            const int fc = pre_to_bfs[pre + 1];
            const int end = ctl->level_off[l + 1] + ctl->level_count[l + 1];
            int nc = 1;
            while (nc < 8 && fc + nc < end && lcp[pre_start[bfs_to_pre[fc + nc]]] >= l) ++nc;
            topo[b] = make_int4(fc, nc, l, 0);
            for (int k = 0; k < nc; ++k) parent[fc + k] = b;
        }
    }
}

// Internal node from its children: box, largest h, mass, centre of mass, and second
// moments about the centre of mass (parallel-axis shifts of the children's).
__device__ void aggregate_node(int p, const int4 tp, double4* nbox_lo, double4* nbox_hi, double4* mom0,
                               double4* mom1, double4* mom2, int2* range, double side, bool mass) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hmax = 0.0, M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    int cnt = 0;
    for (int k = 0; k < tp.y; ++k) {
        const int c = tp.x + k;
        const double4 a = nbox_lo[c], b = nbox_hi[c];
        lo[0] = fmin(lo[0], a.x); lo[1] = fmin(lo[1], a.y); lo[2] = fmin(lo[2], a.z);
        hi[0] = fmax(hi[0], b.x); hi[1] = fmax(hi[1], b.y); hi[2] = fmax(hi[2], b.z);
        hmax = fmax(hmax, a.w);
        if (mass) {
            const double4 m0 = mom0[c];
            M += m0.x;
            sx += m0.x * m0.y; sy += m0.x * m0.z; sz += m0.x * m0.w;
        }
        cnt += range[c].y;
    }
    nbox_lo[p] = make_double4(lo[0], lo[1], lo[2], hmax);
    nbox_hi[p] = make_double4(hi[0], hi[1], hi[2], side);
    range[p] = make_int2(range[tp.x].x, cnt);
    if (!mass) return;
    const double cx = sx / M, cy = sy / M, cz = sz / M;
    double I[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < tp.y; ++k) {
        const int c = tp.x + k;
        const double4 m0 = mom0[c], m1 = mom1[c], m2 = mom2[c];
        const double dx = m0.y - cx, dy = m0.z - cy, dz = m0.w - cz;
        I[0] += m1.x + m0.x * dx * dx; I[1] += m1.y + m0.x * dy * dy; I[2] += m1.z + m0.x * dz * dz;
        I[3] += m2.x + m0.x * dx * dy; I[4] += m2.y + m0.x * dx * dz; I[5] += m2.z + m0.x * dy * dz;
    }
    mom0[p] = make_double4(M, cx, cy, cz);
    mom1[p] = make_double4(I[0], I[1], I[2], I[0] + I[1] + I[2]);
    mom2[p] = make_double4(I[3], I[4], I[5], 0.0);
}

// Leaf geometry and moments from its particles [s, s + c).
__device__ void leaf_node(int b, int s, int c, const double4* __restrict__ pos4, const double* __restrict__ m,
                          double4* nbox_lo, double4* nbox_hi, double4* mom0, double4* mom1, double4* mom2,
                          int2* range, double side, bool mass) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hmax = 0.0, M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    const int e = s + c;
    if (!mass) {
#pragma unroll 4
        for (int j = s; j < e; ++j) {
            const double4 p = pos4[j];
            lo[0] = fmin(lo[0], p.x); lo[1] = fmin(lo[1], p.y); lo[2] = fmin(lo[2], p.z);
            hi[0] = fmax(hi[0], p.x); hi[1] = fmax(hi[1], p.y); hi[2] = fmax(hi[2], p.z);
            hmax = fmax(hmax, p.w);
        }
        nbox_lo[b] = make_double4(lo[0], lo[1], lo[2], hmax);
        nbox_hi[b] = make_double4(hi[0], hi[1], hi[2], side);
        range[b] = make_int2(s, c);
        return;
    }
#pragma unroll 4
    for (int j = s; j < e; ++j) {
        const double4 p = pos4[j];
        const double mj = m[j];
        lo[0] = fmin(lo[0], p.x); lo[1] = fmin(lo[1], p.y); lo[2] = fmin(lo[2], p.z);
        hi[0] = fmax(hi[0], p.x); hi[1] = fmax(hi[1], p.y); hi[2] = fmax(hi[2], p.z);
        hmax = fmax(hmax, p.w);
        M += mj; sx += mj * p.x; sy += mj * p.y; sz += mj * p.z;
    }
    const double cx = sx / M, cy = sy / M, cz = sz / M;
    double I[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
    for (int j = s; j < e; ++j) {
        const double4 p = pos4[j];
        const double mj = m[j];
        const double dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
        I[0] += mj * dx * dx; I[1] += mj * dy * dy; I[2] += mj * dz * dz;
        I[3] += mj * dx * dy; I[4] += mj * dx * dz; I[5] += mj * dy * dz;
    }
    nbox_lo[b] = make_double4(lo[0], lo[1], lo[2], hmax);
    nbox_hi[b] = make_double4(hi[0], hi[1], hi[2], side);
    mom0[b] = make_double4(M, cx, cy, cz);
    mom1[b] = make_double4(I[0], I[1], I[2], I[0] + I[1] + I[2]);
    mom2[b] = make_double4(I[3], I[4], I[5], 0.0);
    range[b] = make_int2(s, c);
}

struct MomArgs {
    const DevCtl* ctl;
    int batched;
    int mass;  // build masses and moments too (gravity on), else only boxes, h_max and ranges
    const u64* key;
    const int4* topo;
    const double4* pos4;
    const double* m;
    double4 *nbox_lo, *nbox_hi, *mom0, *mom1, *mom2;
    int2* range;
};

// Node b: a leaf from its particles, an internal node from its (finished) children.
__device__ __forceinline__ void node_moments(const MomArgs& A, int b) {
    const int4 tp = A.topo[b];
    const int s = tp.w ? tp.x : A.range[tp.x].x;
    const int seg = A.batched ? (int)((A.key[s] >> 54) & 511ull) : 0;
    const double side = ldexp(A.ctl->side[seg], -tp.z);
    if (tp.w)
        leaf_node(b, tp.x, tp.y, A.pos4, A.m, A.nbox_lo, A.nbox_hi, A.mom0, A.mom1, A.mom2, A.range, side, A.mass);
    else
        aggregate_node(b, tp, A.nbox_lo, A.nbox_hi, A.mom0, A.mom1, A.mom2, A.range, side, A.mass);
}

// Every node at level >= cut: one wavefront per level-cut cell finishes its whole subtree
// bottom-up.  A subtree's nodes at each level are one contiguous run in breadth-first
// order (from the first child of its first internal node to the last child of its last
// internal node), so the runs are found top-down, then the levels are done deepest first
// with the wavefront's own results as inputs.  The levels between the cut and the top
// block go one launch each; large sets cut deeper, so that centrally concentrated ones do
// not leave a few waves with very deep subtrees.  The top block is one workgroup on one CU:
// it takes levels 3 .. 0 only, since a sparse outer shell (the polytrope's) puts thousands of
// nodes and leaves at level 4, which a grid-wide launch handles faster.
constexpr int TOP_LEVELS = 4;
static int subtree_cut(int n) { return n >= (1 << 21) ? 9 : 6; }
__global__ void __launch_bounds__(64) k_subtree_moments(MomArgs A, int cut) {
    __shared__ int run_lo[MAX_LEVEL + 1], run_hi[MAX_LEVEL + 1];
    const int lane = lane_id();
    const int nroot = A.ctl->level_count[cut], r0 = A.ctl->level_off[cut];
    for (int ri = blockIdx.x; ri < nroot; ri += gridDim.x) {
        int lo = r0 + ri, hi = lo, deep = cut;
        if (lane == 0) {
            run_lo[cut] = lo;
            run_hi[cut] = hi;
        }
        for (int l = cut; l < MAX_LEVEL; ++l) {
            int first = -1, last = -1;
            for (int k0 = lo; k0 <= hi && first < 0; k0 += 64) {  // first internal node
                const int k = k0 + lane;
                const u64 bl = __ballot(k <= hi && !A.topo[k].w);
                if (bl) first = k0 + __ffsll((long long)bl) - 1;
            }
            if (first < 0) break;
            for (int k1 = hi; k1 >= lo && last < 0; k1 -= 64) {  // last internal node
                const int k = k1 - lane;
                const u64 bl = __ballot(k >= lo && !A.topo[k].w);
                if (bl) last = k1 - (__ffsll((long long)bl) - 1);
            }
            const int4 tf = A.topo[first], tl = A.topo[last];
            lo = tf.x;
            hi = tl.x + tl.y - 1;
            deep = l + 1;
            if (lane == 0) {
                run_lo[deep] = lo;
                run_hi[deep] = hi;
            }
        }
        __syncthreads();
        for (int l = deep; l >= cut; --l) {
            const int a = run_lo[l], e = run_hi[l];
            for (int k = a + lane; k <= e; k += 64) node_moments(A, k);
            __syncthreads();
        }
    }
}

// Nodes of one level (the level below it complete), one node per thread.
__global__ void __launch_bounds__(256) k_level_moments(MomArgs A, int level) {
    const int b0 = A.ctl->level_off[level], nb = A.ctl->level_count[level];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += gridDim.x * blockDim.x) node_moments(A, b0 + k);
}

// Levels TOP_LEVELS - 1 .. 0 in one workgroup, a barrier between levels (their nodes are few).
__global__ void __launch_bounds__(1024) k_top_moments(MomArgs A) {
    for (int level = TOP_LEVELS - 1; level >= 0; --level) {
        const int b0 = A.ctl->level_off[level], nb = A.ctl->level_count[level];
        for (int k = threadIdx.x; k < nb; k += blockDim.x) node_moments(A, b0 + k);
        __syncthreads();
    }
}

static int grid_cap(int n, int bs, int cap) {
    int g = (n + bs - 1) / bs;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

void build_octree(hipStream_t s, const DevPtrs& d, const Dims& dm) {
    const int n = dm.n;
    if (n <= 0) return;
    auto levels = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((n + TB - 1) / TB), dim3(TB), 0, s, d.key_a, n, dm.leaf_size, dm.min_level, d.lcp,
                           d.lvl, d.scan_in, d.ctl, d.gflag);
    };
    switch (dm.leaf_size) {  // the autotuner's leaf sizes and the node-node scheme's 64
        case 8: levels(k_leaf_levels<8>); break;
        case 12: levels(k_leaf_levels<12>); break;
        case 16: levels(k_leaf_levels<16>); break;
        case 24: levels(k_leaf_levels<24>); break;
        case 32: levels(k_leaf_levels<32>); break;
        case 64: levels(k_leaf_levels<64>); break;
        default: levels(k_leaf_levels<0>); break;
    }
    scan_u64(s, d.scan_in, d.scan_out, n, d.scan_tmp);
    hipLaunchKernelGGL(k_emit_nodes, dim3(grid_cap(n, 256, 512)), dim3(256), 0, s, n, d.lcp, d.lvl, d.scan_out,
                       d.pre_level, d.pre_leaf, d.pre_start, d.leaf_start, d.leaf_pre, d.ctl, dm.node_cap);
    const int tiles_cap = grid_cap(dm.node_cap, LS_TILE, 1024);
    hipLaunchKernelGGL(k_lsort_hist, dim3(tiles_cap), dim3(LS_THREADS), 0, s, d.ctl, d.pre_level, d.lsort_hist);
    hipLaunchKernelGGL(k_lsort_scan, dim3(24), dim3(64), 0, s, d.ctl, d.lsort_hist);
    hipLaunchKernelGGL(k_lsort_scatter, dim3(tiles_cap), dim3(LS_THREADS), 0, s, d.ctl, d.pre_level, d.lsort_hist,
                       d.pre_to_bfs, d.bfs_to_pre);
    const int g = grid_cap(dm.node_cap, 256, 2048);
    hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, d.ctl, d.pre_level, d.pre_leaf, d.pre_start,
                       d.pre_to_bfs, d.bfs_to_pre, d.lcp, d.scan_out, d.leaf_start, d.topo, d.parent, d.counter,
                       d.range);
    // moments: subtrees below the cut, then the levels between, then the top levels
    const int cut = subtree_cut(n);
    const MomArgs A{d.ctl, dm.batched, dm.mass_moments, d.key_a, d.topo, d.pos4, d.m,
                    d.nbox_lo, d.nbox_hi, d.mom0, d.mom1, d.mom2, d.range};
    hipLaunchKernelGGL(k_subtree_moments, dim3(grid_cap(n, 64, 8192)), dim3(64), 0, s, A, cut);
    for (int lv = cut - 1; lv >= TOP_LEVELS; --lv)
        hipLaunchKernelGGL(k_level_moments, dim3(grid_cap(n / 2 + 1, 256, 256)), dim3(256), 0, s, A, lv);
    hipLaunchKernelGGL(k_top_moments, dim3(1), dim3(1024), 0, s, A);
    // target groups: cells of at most 4 * group_size particles, cut into runs of group_size
    const int gcap = 4 * dm.group_size;
    hipLaunchKernelGGL(k_group_starts, dim3(g), dim3(256), 0, s, d.ctl, gcap, dm.group_size, dm.min_level, d.topo,
                       d.parent, d.range, d.gflag, d.gsize);
    scan_u32_total(s, d.gflag, d.gscan, n, d.scan_tmp);
    hipLaunchKernelGGL(k_emit_groups, dim3((n + 255) / 256), dim3(256), 0, s, n, dm.batched, d.ctl, d.gflag, d.gscan,
                       d.gsize, d.key_a, d.seg_root_rank, d.group);
}

// Export (test path): node keys etc. in breadth-first order.
__global__ void k_tree_export(const DevCtl* __restrict__ ctl, int n, const u64* __restrict__ key,
                              const int4* __restrict__ topo,
                              const int2* __restrict__ range, u64* okey, int32_t* olevel, int32_t* oleaf,
                              int64_t* ostart, int64_t* ocount) {
    const int nn = ctl->n_nodes;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nn; b += gridDim.x * blockDim.x) {
        const int4 t = topo[b];
        int2 r = range[b];
        if (r.x < 0 || r.x >= n) r.x = 0;
        const int l = t.z;
        const u64 body = key[r.x] & 0x7fffffffffffffffull;
        const u64 digits = l == 0 ? 0ull : (body >> (3 * (MAX_LEVEL - l)));
        if (okey) okey[b] = (1ull << (3 * l)) | digits;
        if (olevel) olevel[b] = l;
        if (oleaf) oleaf[b] = t.w;
        if (ostart) ostart[b] = r.x;
        if (ocount) ocount[b] = r.y;
    }
}

void launch_tree_export(hipStream_t s, const DevPtrs& d, const Dims& dm, u64* key, int32_t* level, int32_t* leaf,
                        int64_t* start, int64_t* count) {
    hipLaunchKernelGGL(k_tree_export, dim3(grid_cap(dm.node_cap, 256, 2048)), dim3(256), 0, s, d.ctl, dm.n, d.key_a,
                       d.topo, d.range, key, level, leaf, start, count);
}
