// Octree self-gravity (Sec. 2.2.2 of arXiv:2007.03097, eq. (10), with Plummer softening
// and quadrupole moments).
//
// One wavefront per target group, two targets per lane.  The wide walk tests up to 64 nodes at once against the
// group's box: a cell B is accepted for the whole group when its particle box does not touch
// the group box and b_B < theta d, b_B being the distance from B's centre of mass to the
// farthest corner of its particle box (B's radius about the centre of mass) and d the
// distance from the centre of mass to the group box (theta = 0 opens everything: the exact
// direct sum).  Accepted
// cells act through the second-order expansion of the softened potential about their
// centre of mass (monopole + quadrupole; the dipole vanishes there):
//   phi += -G [M/s + (3/2) R.I.R/s^5 - (1/2) tr(I)/s^3]
//   g   +=  G [-M R/s^3 + 3 I.R/s^5 - (15/2) (R.I.R) R/s^7 + (3/2) tr(I) R/s^5]
// with R = r_a - R_B, s^2 = |R|^2 + eps^2, I = sum m y y^T about R_B.  Unaccepted leaves
// contribute softened particle sums with the target itself skipped.  Cell and leaf lists
// live in LDS and are evaluated whenever they fill, so the walk needs no global scratch;
// the evaluation stages cell moments (32 at a time in FP64, 64 in FP32C) and leaf particles
// (64 at a time) through LDS.
#include "common.h"

constexpr int GW_STACK = 768;
constexpr int GW_CELLS = 448;
constexpr int GW_LEAVES = 256;
// Stack headroom kept free of wide rounds: popping one entry at a time (depth first), the
// stack grows by at most 7 per tree level below the popped node, so rounds of 64 entries
// stop DFS_HEADROOM entries short of the top and single-entry rounds cannot overflow it.
constexpr int DFS_HEADROOM = 7 * MAX_LEVEL + 8;
static_assert(GW_STACK > 2 * DFS_HEADROOM, "room for wide rounds above the headroom");

// LDS staging of one evaluation: cell moments in the cell phase, particles in the leaf phase.
// FP32C stages FP32 records, 64 cells per round; FP64 stages 32 cells of 96 bytes per round.
// Either way the walk's LDS stays near 10 KB per workgroup (16 workgroups per CU).
template <bool FP32C>
struct GravStage;
template <>
struct GravStage<false> {
    union {
        struct {
            // (M, com), (3 Ixx, 3 Iyy, 3 Izz, 3/2 tr I), (3 Ixy, 3 Ixz, 3 Iyz, 1/2 tr I)
            double4 c0[32], c1[32], c2[32];
        } cell;
        struct {
            double4 pm[64];  // (x, y, z, m)
            int src[64];     // particle index (self test without softening)
        } part;
    };
    int loff[GW_LEAVES + 1];  // particle offsets of the staged leaves
};
template <>
struct GravStage<true> {
    union {
        struct {             // positions as offsets from the group origin
            float4 c0[64], c1[64], c2[64];
        } cellf;
        struct {
            float4 pm[64];
            int src[64];
        } partf;
        struct {
            double4 pm[64];
            int src[64];
        } part;
    };
    int loff[GW_LEAVES + 1];
};

// Kahan-compensated FP32 sum of FP32 partial sums (one add per staged tile).
struct KahanF {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// Per-target accumulators: FP64 sums, or FP32 sums of one staged tile (t*) that enter
// Kahan-compensated FP32 accumulators (k*) once per tile.
struct TargetSums {
    double gx = 0, gy = 0, gz = 0, ph = 0;
    float tx = 0, ty = 0, tz = 0, tph = 0;
    KahanF kx, ky, kz, kp;
    __device__ __forceinline__ void flush_tile() {
        kx.add(tx); ky.add(ty); kz.add(tz); kp.add(tph);
        tx = ty = tz = tph = 0.0f;
    }
};

// Monopole + quadrupole of a staged cell, with the expansion's constants folded into the
// record at staging: a = (M, com), b = (3 Ixx, 3 Iyy, 3 Izz, 3/2 tr I), d = (3 Ixy, 3 Ixz,
// 3 Iyz, 1/2 tr I).  With Q = 3 I: g += -M R/s^3 + Q.R/s^5 - (5/2) (R.Q.R) R/s^7 + (3/2) tr(I) R/s^5
// and phi -= M/s + (1/2) R.Q.R/s^5 - (1/2) tr(I)/s^3.
template <bool PH = true>
__device__ __forceinline__ void cell_term(const double4 me, const double4 a, const double4 b, const double4 d,
                                          double e2, TargetSums& S) {
    const double Rx = me.x - a.y, Ry = me.y - a.z, Rz = me.z - a.w;
    const double QRx = fma(b.x, Rx, fma(d.x, Ry, d.y * Rz));
    const double QRy = fma(d.x, Rx, fma(b.y, Ry, d.z * Rz));
    const double QRz = fma(d.y, Rx, fma(d.z, Ry, b.z * Rz));
    const double RQR = fma(Rx, QRx, fma(Ry, QRy, Rz * QRz));
    const double s2 = fma(Rx, Rx, fma(Ry, Ry, fma(Rz, Rz, e2)));
    const double i1 = rsq_nr1(s2);
    const double i2 = i1 * i1, i3 = i1 * i2, i5 = i3 * i2, i7 = i5 * i2;
    const double cR = fma(b.w, i5, fma(-2.5 * RQR, i7, -a.x * i3));
    S.gx = fma(cR, Rx, fma(i5, QRx, S.gx));
    S.gy = fma(cR, Ry, fma(i5, QRy, S.gy));
    S.gz = fma(cR, Rz, fma(i5, QRz, S.gz));
    if constexpr (PH) S.ph -= fma(a.x, i1, fma(0.5 * RQR, i5, -d.w * i3));
}

// Softened particle term of source sb = (x, y, z, m).
template <bool FP32C, bool PH = true>
__device__ __forceinline__ void part_term(const double4 me, const double4 sb, double e2, TargetSums& S) {
    if (!FP32C) {
        const double dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
        const double s2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, e2)));
        const double i1 = rsq_nr1(s2);
        const double mi3 = sb.w * i1 * i1 * i1;
        S.gx = fma(-mi3, dx, S.gx);
        S.gy = fma(-mi3, dy, S.gy);
        S.gz = fma(-mi3, dz, S.gz);
        if constexpr (PH) S.ph = fma(-sb.w, i1, S.ph);
    } else {
        const float dx = (float)(me.x - sb.x), dy = (float)(me.y - sb.y), dz = (float)(me.z - sb.z);
        const float s2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, (float)e2)));
        const float i1 = __builtin_amdgcn_rsqf(s2);
        const float mb = (float)sb.w;
        const float mi3 = mb * i1 * i1 * i1;
        S.tx = fmaf(-mi3, dx, S.tx);
        S.ty = fmaf(-mi3, dy, S.ty);
        S.tz = fmaf(-mi3, dz, S.tz);
        if constexpr (PH) S.tph = fmaf(-mb, i1, S.tph);
    }
}

// FP32C forms on group-origin offsets: the target and the cell's centre of mass (or the
// source particle) are FP32 offsets from the group's first target, each formed in FP64 and
// rounded once, so one FP32 subtraction gives R (its error is within u (|r_a - o| + |R_B - o|),
// small against |R| for accepted cells, and softened for near particle pairs).
template <bool PH = true>
__device__ __forceinline__ void cell_term_f(const float4 me, const float4 a, const float4 b, const float4 d, float e2,
                                            TargetSums& S) {
    const float Rx = me.x - a.y, Ry = me.y - a.z, Rz = me.z - a.w;
    const float QRx = fmaf(b.x, Rx, fmaf(d.x, Ry, d.y * Rz));
    const float QRy = fmaf(d.x, Rx, fmaf(b.y, Ry, d.z * Rz));
    const float QRz = fmaf(d.y, Rx, fmaf(d.z, Ry, b.z * Rz));
    const float RQR = fmaf(Rx, QRx, fmaf(Ry, QRy, Rz * QRz));
    const float s2 = fmaf(Rx, Rx, fmaf(Ry, Ry, fmaf(Rz, Rz, e2)));
    const float i1 = __builtin_amdgcn_rsqf(s2);
    const float i2 = i1 * i1, i3 = i1 * i2, i5 = i3 * i2, i7 = i5 * i2;
    const float cR = fmaf(b.w, i5, fmaf(-2.5f * RQR, i7, -a.x * i3));
    S.tx = fmaf(cR, Rx, fmaf(i5, QRx, S.tx));
    S.ty = fmaf(cR, Ry, fmaf(i5, QRy, S.ty));
    S.tz = fmaf(cR, Rz, fmaf(i5, QRz, S.tz));
    if constexpr (PH) S.tph -= fmaf(a.x, i1, fmaf(0.5f * RQR, i5, -d.w * i3));
}

template <bool PH = true>
__device__ __forceinline__ void part_term_f(const float4 me, const float4 sb, float e2, TargetSums& S) {
    const float dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
    const float s2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, e2)));
    const float i1 = __builtin_amdgcn_rsqf(s2);
    const float mi3 = sb.w * i1 * i1 * i1;
    S.tx = fmaf(-mi3, dx, S.tx);
    S.ty = fmaf(-mi3, dy, S.ty);
    S.tz = fmaf(-mi3, dz, S.tz);
    if constexpr (PH) S.tph = fmaf(-sb.w, i1, S.tph);
}

// Two targets per lane: tp and tp + TP (TP = group_size / 2); the P = 64 / TP lanes with
// the same tp split every staged tile, so each LDS read of a cell or particle feeds two
// evaluations.
struct GravTargets {
    double4 a, b;
    float4 fa, fb;  // FP32C: offsets from the group origin o
    double o[3];
    int qa, qb;
    bool va, vb;
    int tp, phi, TP, P;
};

// Accepted cells (monopole + quadrupole) for the lane's targets, staged CS at a time (one
// lane loads one cell).
// A compile-time flag passed as a value, to select a template from a run-time branch.
template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

template <bool FP32C>
__device__ void eval_cells(int ncell, const int* cells, GravStage<FP32C>& St, const double4* __restrict__ mom0,
                           const double4* __restrict__ mom1, const double4* __restrict__ mom2, const GravTargets& T,
                           double e2, bool phi, TargetSums& A, TargetSums& B) {
    const int lane = lane_id();
    const bool any = T.va || T.vb;
    constexpr int CS = FP32C ? 64 : 32;  // cells staged per round
    for (int k0 = 0; k0 < ncell; k0 += CS) {
        __syncthreads();
        if (lane < CS && k0 + lane < ncell) {
            const int c = cells[k0 + lane];
            const double4 c0 = mom0[c], c1 = mom1[c], c2 = mom2[c];
            if constexpr (FP32C) {
                St.cellf.c0[lane] = make_float4((float)c0.x, (float)(c0.y - T.o[0]), (float)(c0.z - T.o[1]),
                                                (float)(c0.w - T.o[2]));
                St.cellf.c1[lane] = make_float4((float)(3.0 * c1.x), (float)(3.0 * c1.y), (float)(3.0 * c1.z),
                                                (float)(1.5 * c1.w));
                St.cellf.c2[lane] = make_float4((float)(3.0 * c2.x), (float)(3.0 * c2.y), (float)(3.0 * c2.z),
                                                (float)(0.5 * c1.w));
            } else {  // the expansion's constants folded in (see cell_term)
                St.cell.c0[lane] = c0;
                St.cell.c1[lane] = make_double4(3.0 * c1.x, 3.0 * c1.y, 3.0 * c1.z, 1.5 * c1.w);
                St.cell.c2[lane] = make_double4(3.0 * c2.x, 3.0 * c2.y, 3.0 * c2.z, 0.5 * c1.w);
            }
        }
        __syncthreads();
        const int cn = ncell - k0 < CS ? ncell - k0 : CS;
        if (!any) continue;
        auto run = [&](auto ph) {
            constexpr bool PH = decltype(ph)::value;
            if constexpr (FP32C) {
                const float e2f = (float)e2;
                for (int k = T.phi; k < cn; k += T.P) {
                    const float4 a = St.cellf.c0[k], b = St.cellf.c1[k], d = St.cellf.c2[k];
                    cell_term_f<PH>(T.fa, a, b, d, e2f, A);
                    cell_term_f<PH>(T.fb, a, b, d, e2f, B);
                }
                A.flush_tile();
                B.flush_tile();
            } else {
                for (int k = T.phi; k < cn; k += T.P) {
                    const double4 a = St.cell.c0[k], b = St.cell.c1[k], d = St.cell.c2[k];
                    cell_term<PH>(T.a, a, b, d, e2, A);
                    cell_term<PH>(T.b, a, b, d, e2, B);
                }
            }
        };
        if (phi) run(BoolC<true>());
        else run(BoolC<false>());
    }
}

// Particles of the listed leaves, concatenated and staged through LDS 64 at a time (one
// load per lane per round): put(lane, position, mass, index) writes the staged record,
// tile(tn) evaluates each staged tile of tn particles.  leaves[] is overwritten with the
// leaves' first particles.
template <typename Stage, typename Tile, typename Put>
__device__ void stage_leaves_put(int nleaf, int* leaves, Stage& St, const int4* __restrict__ topo,
                                 const double4* __restrict__ pos4, const double* __restrict__ m, Tile&& tile,
                                 Put&& put) {
    const int lane = lane_id();
    int carry = 0;
    for (int j0 = 0; j0 < nleaf; j0 += 64) {  // particle offsets of the leaves
        const int j = j0 + lane;
        int c = 0, st = 0;
        if (j < nleaf) {
            const int4 tp = topo[leaves[j]];
            st = tp.x;
            c = tp.y;
        }
        const int incl = wave_incl_scan(c);
        __syncthreads();
        if (j < nleaf) {
            leaves[j] = st;
            St.loff[j] = carry + incl - c;
        }
        carry += __shfl(incl, 63, 64);
    }
    __syncthreads();
    const int total = carry;
    for (int p0 = 0; p0 < total; p0 += 64) {
        const int p = p0 + lane;
        __syncthreads();
        if (p < total) {
            int a = 0, b = nleaf - 1;
            while (a < b) {  // largest j with loff[j] <= p
                const int mid = (a + b + 1) >> 1;
                if (St.loff[mid] <= p) a = mid;
                else b = mid - 1;
            }
            const int src = leaves[a] + (p - St.loff[a]);
            put(lane, pos4[src], m[src], src);
        }
        __syncthreads();
        tile(total - p0 < 64 ? total - p0 : 64);
    }
}

// stage_leaves_put with (x, y, z, m) records in FP64.
template <typename Stage, typename Tile>
__device__ void stage_leaves(int nleaf, int* leaves, Stage& St, const int4* __restrict__ topo,
                             const double4* __restrict__ pos4, const double* __restrict__ m, Tile&& tile) {
    stage_leaves_put(nleaf, leaves, St, topo, pos4, m, tile, [&](int lane, const double4& ps, double mass, int src) {
        St.part.pm[lane] = make_double4(ps.x, ps.y, ps.z, mass);
        St.part.src[lane] = src;
    });
}

// Leaves evaluated by softened particle sums (self excluded) for the lane's two targets.
// With softening the self pair is evaluated like any other (it adds no force) and its
// potential term -m_q/eps is taken out by the caller.
template <bool FP32C>
__device__ void eval_leaves(int nleaf, int* leaves, GravStage<FP32C>& St, const int4* __restrict__ topo,
                            const double4* __restrict__ pos4, const double* __restrict__ m, const GravTargets& T,
                            double e2, bool phi, TargetSums& A, TargetSums& B) {
    const bool any = T.va || T.vb;
    const bool soft = e2 > 0.0;
    if constexpr (FP32C) {
        const float e2f = (float)e2;
        auto run = [&](int tn, auto ph) {
            constexpr bool PH = decltype(ph)::value;
            if (soft) {
                for (int j = T.phi; j < tn; j += T.P) {
                    const float4 sb = St.partf.pm[j];
                    part_term_f<PH>(T.fa, sb, e2f, A);
                    part_term_f<PH>(T.fb, sb, e2f, B);
                }
            } else {
                for (int j = T.phi; j < tn; j += T.P) {
                    const float4 sb = St.partf.pm[j];
                    const int s = St.partf.src[j];
                    if (s != T.qa) part_term_f<PH>(T.fa, sb, e2f, A);
                    if (s != T.qb) part_term_f<PH>(T.fb, sb, e2f, B);
                }
            }
        };
        stage_leaves_put(
            nleaf, leaves, St, topo, pos4, m,
            [&](int tn) {
                if (!any) return;
                if (phi) run(tn, BoolC<true>());
                else run(tn, BoolC<false>());
                A.flush_tile();
                B.flush_tile();
            },
            [&](int lane, const double4& ps, double mass, int src) {
                St.partf.pm[lane] = make_float4((float)(ps.x - T.o[0]), (float)(ps.y - T.o[1]), (float)(ps.z - T.o[2]),
                                                (float)mass);
                St.partf.src[lane] = src;
            });
        return;
    }
    auto run = [&](int tn, auto ph) {
        constexpr bool PH = decltype(ph)::value;
        if (soft) {
            for (int j = T.phi; j < tn; j += T.P) {
                const double4 sb = St.part.pm[j];
                part_term<false, PH>(T.a, sb, e2, A);
                part_term<false, PH>(T.b, sb, e2, B);
            }
        } else {
            for (int j = T.phi; j < tn; j += T.P) {
                const double4 sb = St.part.pm[j];
                const int s = St.part.src[j];
                if (s != T.qa) part_term<false, PH>(T.a, sb, e2, A);
                if (s != T.qb) part_term<false, PH>(T.b, sb, e2, B);
            }
        }
    };
    stage_leaves(nleaf, leaves, St, topo, pos4, m, [&](int tn) {
        if (!any) return;
        if (phi) run(tn, BoolC<true>());
        else run(tn, BoolC<false>());
    });
}

// One target per lane: target t of c (lanes t + c ph, ph < P = 64 / c, split the staged
// sources), for targets that fill a wave poorly (the particles of one octree leaf).
struct LaneTarget {
    double4 a;
    int q;
    bool v;
    int ph, P;
};

template <bool FP32C, typename Stage>
__device__ void eval_leaves1(int nleaf, int* leaves, Stage& St, const int4* __restrict__ topo,
                             const double4* __restrict__ pos4, const double* __restrict__ m, const LaneTarget& T,
                             double e2, bool phi, TargetSums& A) {
    const bool soft = e2 > 0.0;
    auto run = [&](int tn, auto ph) {
        constexpr bool PH = decltype(ph)::value;
        if (soft) {
            for (int j = T.ph; j < tn; j += T.P) part_term<FP32C, PH>(T.a, St.part.pm[j], e2, A);
        } else {
            for (int j = T.ph; j < tn; j += T.P)
                if (St.part.src[j] != T.q) part_term<FP32C, PH>(T.a, St.part.pm[j], e2, A);
        }
    };
    stage_leaves(nleaf, leaves, St, topo, pos4, m, [&](int tn) {
        if (!T.v) return;
        if (phi) run(tn, BoolC<true>());
        else run(tn, BoolC<false>());
        if (FP32C) A.flush_tile();
    });
}

// Terms one flush of the lists evaluates: ncell cells and the particles of nleaf leaves, each
// against the group's ng targets (leaves still unstaged), added to the group's running counts
// (the same in every lane).  A group adds them to the pass's counters once, at its end: a
// returnless atomic still holds the wave's next memory wait, and one per flush on two
// addresses shared by the whole grid cost ~12% of the 4M-particle pass.
__device__ __forceinline__ void count_terms(int ncell, int nleaf, const int* leaves, const int4* __restrict__ topo,
                                            int ng, u64& cells, u64& pairs) {
    u64 np = 0;
    for (int i = lane_id(); i < nleaf; i += 64) np += (u64)topo[leaves[i]].y;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) np += __shfl_xor(np, d, 64);
    cells += (u64)ncell * (u64)ng;
    pairs += np * (u64)ng;
}

__global__ void k_zero_grav_counts(DevCtl* ctl) {
    const int s = threadIdx.x;
    if (s < GRAV_SLOTS) {
        ctl->grav_cnt[s][0] = 0;
        ctl->grav_cnt[s][1] = 0;
    }
}

template <bool FP32C>
__device__ void eval_lists(int ncell, int nleaf, const int* cells, int* leaves, GravStage<FP32C>& St,
                           const int4* __restrict__ topo, const double4* __restrict__ mom0,
                           const double4* __restrict__ mom1, const double4* __restrict__ mom2,
                           const double4* __restrict__ pos4, const double* __restrict__ m, const GravTargets& T,
                           double eps, bool phi, TargetSums& A, TargetSums& B) {
    eval_cells<FP32C>(ncell, cells, St, mom0, mom1, mom2, T, eps * eps, phi, A, B);
    eval_leaves<FP32C>(nleaf, leaves, St, topo, pos4, m, T, eps * eps, phi, A, B);
}

template <bool FP32C>
__global__ void __launch_bounds__(64) k_gravity(DevCtl* ctl, const int4* __restrict__ group, int gsz,
                                                const int4* __restrict__ topo, const double4* __restrict__ nbox_lo,
                                                const double4* __restrict__ nbox_hi, const double4* __restrict__ mom0,
                                                const double4* __restrict__ mom1, const double4* __restrict__ mom2,
                                                const double4* __restrict__ pos4, const double* __restrict__ m,
                                                double G, double eps, double theta, int accumulate,
                                                double* __restrict__ gxo, double* __restrict__ gyo,
                                                double* __restrict__ gzo, double* __restrict__ pho,
                                                const double4* __restrict__ vel4, double* __restrict__ deo) {
    __shared__ int stack[GW_STACK];
    __shared__ int cells[GW_CELLS];
    __shared__ int leaves[GW_LEAVES];
    __shared__ GravStage<FP32C> St;
    const int lane = lane_id();
    GravTargets T;
    // the potential is evaluated (and written) unless the step sequence has switched it off:
    // inside a run of steps only the last step's value is read (by the energy diagnostic)
    const bool phi = pho != nullptr && ctl->skip_phi == 0;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
        const int4 g = group[gi];
        // TP target pairs per wave, the fewest (a power of two) that hold the group's targets:
        // the P = 64 / TP lanes of a pair split each staged tile, so a group with few
        // targets keeps every lane busy
        T.TP = 1;
        while (2 * T.TP < g.y && T.TP < (gsz >> 1)) T.TP <<= 1;
        T.P = 64 / T.TP;
        T.tp = lane & (T.TP - 1);
        T.phi = lane / T.TP;
        T.qa = g.x + T.tp;
        T.qb = g.x + T.tp + T.TP;
        T.va = T.tp < g.y;
        T.vb = T.tp + T.TP < g.y;
        T.a = T.va ? pos4[T.qa] : make_double4(0, 0, 0, 0);
        T.b = T.vb ? pos4[T.qb] : make_double4(0, 0, 0, 0);
        if (FP32C) {
            const double4 o = pos4[g.x];
            T.o[0] = o.x;
            T.o[1] = o.y;
            T.o[2] = o.z;
            T.fa = make_float4((float)(T.a.x - o.x), (float)(T.a.y - o.y), (float)(T.a.z - o.z), 0.0f);
            T.fb = make_float4((float)(T.b.x - o.x), (float)(T.b.y - o.y), (float)(T.b.z - o.z), 0.0f);
        }
        double lo[3], hi[3];
        lo[0] = wave_min(fmin(T.va ? T.a.x : INFINITY, T.vb ? T.b.x : INFINITY));
        lo[1] = wave_min(fmin(T.va ? T.a.y : INFINITY, T.vb ? T.b.y : INFINITY));
        lo[2] = wave_min(fmin(T.va ? T.a.z : INFINITY, T.vb ? T.b.z : INFINITY));
        hi[0] = wave_max(fmax(T.va ? T.a.x : -INFINITY, T.vb ? T.b.x : -INFINITY));
        hi[1] = wave_max(fmax(T.va ? T.a.y : -INFINITY, T.vb ? T.b.y : -INFINITY));
        hi[2] = wave_max(fmax(T.va ? T.a.z : -INFINITY, T.vb ? T.b.z : -INFINITY));
        for (int c = 0; c < 3; ++c) {  // the group box in scalar registers
            lo[c] = uniform_d(lo[c]);
            hi[c] = uniform_d(hi[c]);
        }
        const double th2 = theta * theta;
        const u64 lt = lanemask_lt();
        TargetSums A, B;
        const int root = g.z < 0 ? 0 : ctl->level_off[3] + g.z;
        __syncthreads();
        if (lane == 0) stack[0] = root;
        int sp = 1, nc = 0, nl = 0, iters = 0;
        u64 n_cells = 0, n_pairs = 0;
        __syncthreads();
        while (sp > 0) {
            if (++iters > (1 << 22)) {  // bounded: every wave leaves the loop
                if (lane == 0) set_err(ctl, ERR_GRAV_LIST);
                break;
            }
            if (nc + 64 > GW_CELLS || nl + 64 > GW_LEAVES) {
                count_terms(nc, nl, leaves, topo, g.y, n_cells, n_pairs);
                eval_lists<FP32C>(nc, nl, cells, leaves, St, topo, mom0, mom1, mom2, pos4, m, T, eps, phi, A, B);
                nc = nl = 0;
                __syncthreads();
            }
            // pop as many nodes as the stack can take the children of (8 each) while keeping
            // the depth-first headroom; past it, one node per round
            int k = sp < 64 ? sp : 64;
            const int room = (GW_STACK - DFS_HEADROOM - sp) / 8;
            if (k > room) k = room > 1 ? room : 1;
            const int node = lane < k ? stack[sp - k + lane] : -1;
            __syncthreads();
            sp -= k;
            int kind = 0;  // 1 = accepted cell, 2 = leaf to open, 3 = open children
            int4 tp = make_int4(0, 0, 0, 0);
            if (node >= 0) {
                tp = topo[node];
                const double4 a = nbox_lo[node], b = nbox_hi[node], m0 = mom0[node];
                const double com[3] = {m0.y, m0.z, m0.w};
                double d2 = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double gp = com[c] < lo[c] ? lo[c] - com[c] : (com[c] > hi[c] ? com[c] - hi[c] : 0.0);
                    d2 += gp * gp;
                }
                const bool apart =
                    a.x > hi[0] || b.x < lo[0] || a.y > hi[1] || b.y < lo[1] || a.z > hi[2] || b.z < lo[2];
                const double ux = fmax(com[0] - a.x, b.x - com[0]), uy = fmax(com[1] - a.y, b.y - com[1]),
                             uz = fmax(com[2] - a.z, b.z - com[2]);
                const double b2 = (ux * ux + uy * uy) + uz * uz;  // radius^2 about the centre of mass
                if (apart && b2 < th2 * d2) kind = 1;
                else kind = tp.w ? 2 : 3;
            }
            const u64 bc = __ballot(kind == 1), bl = __ballot(kind == 2);
            if (kind == 1) cells[nc + __popcll(bc & lt)] = node;
            if (kind == 2) leaves[nl + __popcll(bl & lt)] = node;
            nc += __popcll(bc);
            nl += __popcll(bl);
            const int nch = kind == 3 ? tp.y : 0;
            const int incl = wave_incl_scan(nch);
            const int tot = __shfl(incl, 63, 64);
            if (sp + tot > GW_STACK) {
                if (lane == 0) set_err(ctl, ERR_GRAV_LIST);
                break;
            }
            for (int j = 0; j < nch; ++j) stack[sp + incl - nch + j] = tp.x + j;
            sp += tot;
            __syncthreads();
        }
        __syncthreads();
        count_terms(nc, nl, leaves, topo, g.y, n_cells, n_pairs);
        eval_lists<FP32C>(nc, nl, cells, leaves, St, topo, mom0, mom1, mom2, pos4, m, T, eps, phi, A, B);
        // per target: lanes tp + TP*phi combine in a fixed butterfly order
        double r[8];
        r[0] = FP32C ? A.kx.value() : A.gx;
        r[1] = FP32C ? A.ky.value() : A.gy;
        r[2] = FP32C ? A.kz.value() : A.gz;
        r[3] = FP32C ? A.kp.value() : A.ph;
        r[4] = FP32C ? B.kx.value() : B.gx;
        r[5] = FP32C ? B.ky.value() : B.gy;
        r[6] = FP32C ? B.kz.value() : B.gz;
        r[7] = FP32C ? B.kp.value() : B.ph;
#pragma unroll
        for (int i = 0; i < 8; ++i) r[i] = G * lanes_sum_d(r[i], T.TP);
        if (T.phi == 0) {
            for (int s = 0; s < 2; ++s) {
                if (!(s ? T.vb : T.va)) continue;
                const int q = s ? T.qb : T.qa;
                double gx = r[4 * s], gy = r[4 * s + 1], gz = r[4 * s + 2], ph = r[4 * s + 3];
                if (eps > 0.0) {  // take out the self pair's potential term (see eval_lists)
                    const double e2 = eps * eps;
                    const double is = FP32C ? (double)__builtin_amdgcn_rsqf((float)e2) : rsq_nr1(e2);
                    ph += G * (m[q] * is);
                }
                if (accumulate) {
                    gxo[q] += gx;
                    gyo[q] += gy;
                    gzo[q] += gz;
                    if (deo) {  // thermokinetic form: the work of gravity on e = u + v^2/2
                        const double4 v = vel4[q];
                        deo[q] += fma(v.x, gx, fma(v.y, gy, v.z * gz));
                    }
                } else {
                    gxo[q] = gx;
                    gyo[q] = gy;
                    gzo[q] = gz;
                }
                if (phi) pho[q] = ph;
            }
        }
        if (lane == 0) {  // last, so that no later memory wait of the group holds for it
            u64* slot = ctl->grav_cnt[gi & (GRAV_SLOTS - 1)];
            atomicAdd(&slot[0], n_cells);
            atomicAdd(&slot[1], n_pairs);
        }
    }
}

void launch_gravity(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double G, double eps, double theta,
                    int accumulate, int thermo) {
    if (dm.n <= 0) return;
    double* gx = accumulate ? d.ax : d.gx;
    double* gy = accumulate ? d.ay : d.gy;
    double* gz = accumulate ? d.az : d.gz;
    double* de = (accumulate && thermo) ? d.du : nullptr;
    hipLaunchKernelGGL(k_zero_grav_counts, dim3(1), dim3(64), 0, s, d.ctl);
    if (fp32c)
        hipLaunchKernelGGL(k_gravity<true>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size, d.topo,
                           d.nbox_lo, d.nbox_hi, d.mom0, d.mom1, d.mom2, d.pos4, d.m, G, eps, theta, accumulate, gx, gy,
                           gz, d.phi, d.vel4, de);
    else
        hipLaunchKernelGGL(k_gravity<false>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size, d.topo,
                           d.nbox_lo, d.nbox_hi, d.mom0, d.mom1, d.mom2, d.pos4, d.m, G, eps, theta, accumulate, gx, gy,
                           gz, d.phi, d.vel4, de);
}

// ---------------------------------------------------------------------------------------
// Symmetric node-node gravity: the paper's own scheme (Sec. 2.2.2, eq. (10), after Dehnen
// 2000).
//
// Interaction set: the mutual recursion over node pairs.  A node paired with itself splits
// into its children's self pairs and every unordered pair of children (a leaf sums its
// particle pairs).  A pair (A, B) of distinct nodes is one node-node term when the opening
// test accepts it; else every particle pair when both are leaves; else the larger node
// (lower level; on equal levels the one whose particles come first in key order) is split,
// unless it is a leaf, in which case the other one is.
//
// Opening test: every octree cell (the cells of the key quantisation) lies inside the
// sphere of radius (sqrt 3 / 2) side about its centre; (A, B) is accepted when
// r_A + r_B < theta |c_A - c_B|.  In integer units of half the finest cell this reads
// 3 T^2 < 4 theta^2 |D|^2 with T = 2 (s_A + s_B) and D = 2 (c_A - c_B), so every decision is
// exact and independent of rounding.  theta = 0 accepts nothing: the direct sum.
//
// Node-node term: first order in the Taylor expansion of the potential about each centre
// of mass, with monopole sources.  Node Y acts on node X through g = -G M_Y R / s^3 at R_X
// (R = R_X - R_Y, s^2 = |R|^2 + eps^2), constant across X, and the potential
// -G M_Y / s - g . (r - R_X).  R flips sign bit for bit between the two directions of a
// pair, so the forces two nodes exert on each other are opposite and central: linear and
// angular momentum are conserved up to rounding.
//
// GPU form: every leaf of the tree is a target of one wavefront, which replays the part of
// the recursion that involves the leaf's ancestors X_0 (root) .. X_D (the leaf): each self
// pair (X_e, X_e) yields the pairs (X_e+1, C) for the other children C of X_e, and a pair
// (X_e, Y) either ends (term or particle pairs), moves down the path (X split) or fans out
// over Y's children.  Every node-node term of an ancestor is evaluated once per leaf below
// it -- no scatter, no atomics, a fixed summation order.  The lanes evaluate 64 accepted
// pairs at a time (one each) and sum the constant fields across the wave at the end;
// the particle pairs of unaccepted leaf pairs go through eval_leaves1, one target per lane
// (a leaf fills a wave poorly; 64 / c lanes share each of its c targets).  The
// potential's linear part is referred to the leaf's centre of mass.
constexpr int FM_STACK = 672;
constexpr int FM_TERMS = 192;
constexpr int FM_LEAVES = 192;
constexpr int FM_TARGETS = 64;    // targets per pass over a leaf (one per lane)
static_assert(7 * MAX_LEVEL + DFS_HEADROOM <= FM_STACK, "the initial pairs of a path and the headroom fit");

// LDS staging of the particle sums (the node-node walk has no cell tiles).
struct FmmStage {
    struct {
        double4 pm[64];  // (x, y, z, m)
        int src[64];     // particle index (self test without softening)
    } part;
    int loff[FM_LEAVES + 1];  // particle offsets of the staged leaves
};

struct FmmPath {
    double4 com[MAX_LEVEL + 1];  // (M, centre of mass) of the ancestor at each depth
    int4 topo[MAX_LEVEL + 1];    // its topology record
    int node[MAX_LEVEL + 1];
    int start[MAX_LEVEL + 1];    // its first particle (key order)
    int cell[MAX_LEVEL + 1][3];  // its integer cell coordinates at its level
};

// Integer coordinates of the cell of every node: its first particle, quantised as for the
// keys and truncated to the node's level; packed 21 bits per axis into the free fourth
// component of mom2 (the walk then reads them with the node's topology, not after it).
__global__ void __launch_bounds__(256) k_fmm_cells(const DevCtl* __restrict__ ctl, const int4* __restrict__ topo,
                                                    const int2* __restrict__ range, const double4* __restrict__ pos4,
                                                    double4* mom2) {
    const double lo[3] = {ctl->box[0], ctl->box[1], ctl->box[2]};
    const double S = ctl->scale[0];
    const u32 top = (1u << MAX_LEVEL) - 1u;
    const int nn = ctl->n_nodes;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nn; b += gridDim.x * blockDim.x) {
        const double4 p = pos4[range[b].x];
        const int sh = MAX_LEVEL - topo[b].z;
        const u64 c = (u64)(quantise(p.x, lo[0], S, top) >> sh) | ((u64)(quantise(p.y, lo[1], S, top) >> sh) << 21) |
                      ((u64)(quantise(p.z, lo[2], S, top) >> sh) << 42);
        mom2[b].w = __longlong_as_double((long long)c);
    }
}

__device__ __forceinline__ void fmm_unpack(u64 c, int* v) {
    v[0] = (int)(c & 0x1fffff);
    v[1] = (int)((c >> 21) & 0x1fffff);
    v[2] = (int)(c >> 42);
}

__device__ __forceinline__ bool fmm_accept(int la, const int* ca, int lb, const int* cb, double th4) {
    const long long T = (1ll << (MAX_LEVEL - la + 1)) + (1ll << (MAX_LEVEL - lb + 1));
    long long D2 = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const long long a = (2ll * ca[d] + 1) << (MAX_LEVEL - la);
        const long long b = (2ll * cb[d] + 1) << (MAX_LEVEL - lb);
        D2 += (a - b) * (a - b);
    }
    return 3.0 * (double)(T * T) < th4 * (double)D2;
}

// Accepted pairs (tnode[k], depth tdep[k]): lane k evaluates pair k, k + 64, ... and keeps
// its own partial sums of the field (fg) and of the potential referred to the leaf's
// centre of mass (fc); the caller sums them across the wave.
template <bool PH>
__device__ __forceinline__ void fmm_eval_terms(int nt, const int* tnode, const unsigned char* tdep, const FmmPath& P,
                                               int D, const double4* __restrict__ mom0, double e2, double& fgx,
                                               double& fgy, double& fgz, double& fc) {
    const double4 cl = P.com[D];
    for (int k = lane_id(); k < nt; k += 64) {
        const double4 cx = P.com[tdep[k]];
        const double4 cy = mom0[tnode[k]];
        const double Rx = cx.y - cy.y, Ry = cx.z - cy.z, Rz = cx.w - cy.w;
        const double s2 = fma(Rx, Rx, fma(Ry, Ry, fma(Rz, Rz, e2)));
        const double i1 = rsq_nr1(s2);
        const double mi1 = cy.x * i1;
        const double mi3 = mi1 * i1 * i1;
        const double gx = -mi3 * Rx, gy = -mi3 * Ry, gz = -mi3 * Rz;
        fgx += gx;
        fgy += gy;
        fgz += gz;
        if constexpr (PH) fc -= mi1 + fma(gx, cl.y - cx.y, fma(gy, cl.z - cx.z, gz * (cl.w - cx.w)));
    }
}

template <bool FP32C>
__global__ void __launch_bounds__(64) k_fmm(DevCtl* ctl, const int* __restrict__ leaf_pre,
                                            const int* __restrict__ pre_to_bfs, const int* __restrict__ parent,
                                            const int4* __restrict__ topo, const int2* __restrict__ range,
                                            const double4* __restrict__ mom0, const double* __restrict__ ncell,
                                            const double4* __restrict__ pos4, const double* __restrict__ m, double G,
                                            double eps, double th4,
                                            int accumulate, double* __restrict__ gxo, double* __restrict__ gyo,
                                            double* __restrict__ gzo, double* __restrict__ pho,
                                            const double4* __restrict__ vel4, double* __restrict__ deo) {
    __shared__ int stk[FM_STACK];
    __shared__ unsigned char sdep[FM_STACK];
    const bool phi = pho != nullptr && ctl->skip_phi == 0;  // as in k_gravity
    __shared__ int tnode[FM_TERMS];
    __shared__ unsigned char tdep[FM_TERMS];
    __shared__ int leaves[FM_LEAVES];
    __shared__ FmmStage St;
    __shared__ FmmPath Pth;
    const int lane = lane_id();
    const double e2 = eps * eps;
    const u64 lt = lanemask_lt();
    int l0, l1, lstep;
    group_range(ctl->n_leaves, l0, l1, lstep);
    for (int li = l0; li < l1; li += lstep) {
        const int L = pre_to_bfs[leaf_pre[li]];
        const int4 tl = topo[L];
        const int D = tl.z;  // one set: the root is at level 0
        __syncthreads();
        if (lane == 0) {
            int b = L;
            for (int e = D; e >= 0; --e) {
                Pth.node[e] = b;
                b = e > 0 ? parent[b] : -1;
            }
        }
        __syncthreads();
        if (lane <= D) {
            const int b = Pth.node[lane];
            const int4 t = topo[b];
            const int st = range[b].x;
            Pth.topo[lane] = t;
            Pth.start[lane] = st;
            Pth.com[lane] = mom0[b];
            fmm_unpack((u64)__double_as_longlong(ncell[4 * b]), Pth.cell[lane]);
        }
        __syncthreads();
        const double4 cl = Pth.com[D];
        for (int t0 = 0; t0 < tl.y; t0 += FM_TARGETS) {
            const int cc = min(FM_TARGETS, tl.y - t0);
            LaneTarget T;
            T.P = 64 / cc;
            T.ph = lane / cc;
            T.q = tl.x + t0 + (lane - T.ph * cc);
            T.v = T.ph < T.P;
            T.a = T.v ? pos4[T.q] : make_double4(0, 0, 0, 0);
            // initial pairs: (X_e+1, C) for every other child C of every ancestor X_e
            const int n0 = lane < D ? Pth.topo[lane].y - 1 : 0;
            const int incl = wave_incl_scan(n0);
            int sp = __shfl(incl, 63, 64);
            if (lane < D) {
                const int4 t = Pth.topo[lane];
                const int nxt = Pth.node[lane + 1];
                int o = incl - n0;
                for (int j = 0; j < t.y; ++j) {
                    const int ch = t.x + j;
                    if (ch != nxt) {
                        stk[o] = ch;
                        sdep[o] = (unsigned char)(lane + 1);
                        ++o;
                    }
                }
            }
            if (lane == 0) leaves[0] = L;  // the leaf's own particle pairs
            int nt = 0, nl = 1, iters = 0;
            TargetSums A;
            double fgx = 0.0, fgy = 0.0, fgz = 0.0, fc = 0.0;
            __syncthreads();
            while (sp > 0) {
                if (++iters > (1 << 22)) {  // bounded: every wave leaves the loop
                    if (lane == 0) set_err(ctl, ERR_GRAV_LIST);
                    break;
                }
                if (nt + 64 > FM_TERMS) {
                    if (phi) fmm_eval_terms<true>(nt, tnode, tdep, Pth, D, mom0, e2, fgx, fgy, fgz, fc);
                    else fmm_eval_terms<false>(nt, tnode, tdep, Pth, D, mom0, e2, fgx, fgy, fgz, fc);
                    nt = 0;
                    __syncthreads();
                }
                if (nl + 64 > FM_LEAVES) {
                    eval_leaves1<FP32C>(nl, leaves, St, topo, pos4, m, T, e2, phi, A);
                    nl = 0;
                    __syncthreads();
                }
                int k = sp < 64 ? sp : 64;  // wide rounds only above the depth-first headroom
                const int room = (FM_STACK - DFS_HEADROOM - sp) / 8;
                if (k > room) k = room > 1 ? room : 1;
                int Y = -1, e = 0;
                if (lane < k) {
                    Y = stk[sp - k + lane];
                    e = sdep[sp - k + lane];
                }
                __syncthreads();
                sp -= k;
                int kind = 0;  // 1 = node-node term, 2 = leaf pair, 3 = split X, 4 = split Y
                int4 ty = make_int4(0, 0, 0, 0);
                if (Y >= 0) {
                    ty = topo[Y];
                    const int sy = range[Y].x;
                    int cy[3];
                    fmm_unpack((u64)__double_as_longlong(ncell[4 * Y]), cy);
                    const int4 tx = Pth.topo[e];
                    if (fmm_accept(tx.z, Pth.cell[e], ty.z, cy, th4)) {
                        kind = 1;
                    } else if (tx.w && ty.w) {
                        kind = 2;
                    } else {
                        bool split_x = tx.z < ty.z || (tx.z == ty.z && Pth.start[e] < sy);
                        if (split_x ? tx.w : ty.w) split_x = !split_x;
                        kind = split_x ? 3 : 4;
                    }
                }
                const u64 bt = __ballot(kind == 1), bl = __ballot(kind == 2);
                if (kind == 1) {
                    const int o = nt + __popcll(bt & lt);
                    tnode[o] = Y;
                    tdep[o] = (unsigned char)e;
                }
                if (kind == 2) leaves[nl + __popcll(bl & lt)] = Y;
                nt += __popcll(bt);
                nl += __popcll(bl);
                const int np = kind == 3 ? 1 : (kind == 4 ? ty.y : 0);
                const int pin = wave_incl_scan(np);
                const int tot = __shfl(pin, 63, 64);
                if (sp + tot > FM_STACK) {
                    if (lane == 0) set_err(ctl, ERR_GRAV_LIST);
                    break;
                }
                if (kind == 3) {
                    stk[sp + pin - 1] = Y;
                    sdep[sp + pin - 1] = (unsigned char)(e + 1);
                } else if (kind == 4) {
                    for (int j = 0; j < np; ++j) {
                        stk[sp + pin - np + j] = ty.x + j;
                        sdep[sp + pin - np + j] = (unsigned char)e;
                    }
                }
                sp += tot;
                __syncthreads();
            }
            __syncthreads();
            if (phi) fmm_eval_terms<true>(nt, tnode, tdep, Pth, D, mom0, e2, fgx, fgy, fgz, fc);
            else fmm_eval_terms<false>(nt, tnode, tdep, Pth, D, mom0, e2, fgx, fgy, fgz, fc);
            eval_leaves1<FP32C>(nl, leaves, St, topo, pos4, m, T, e2, phi, A);
            fgx = lanes_sum_d(fgx, 1);
            fgy = lanes_sum_d(fgy, 1);
            fgz = lanes_sum_d(fgz, 1);
            fc = lanes_sum_d(fc, 1);
            // each target's P partial sums (lanes t + cc ph) combined in phase order
            __syncthreads();
            St.part.pm[lane] = FP32C ? make_double4(A.kx.value(), A.ky.value(), A.kz.value(), A.kp.value())
                                     : make_double4(A.gx, A.gy, A.gz, A.ph);
            __syncthreads();
            if (T.v && T.ph == 0) {
                double4 r = St.part.pm[lane];
                for (int k = 1; k < T.P; ++k) {
                    const double4 o = St.part.pm[lane + k * cc];
                    r.x += o.x;
                    r.y += o.y;
                    r.z += o.z;
                    r.w += o.w;
                }
                {
                    const int q = T.q;
                    const double4 me = T.a;
                    const double lin = fma(fgx, me.x - cl.y, fma(fgy, me.y - cl.z, fgz * (me.z - cl.w)));
                    const double gx = G * (r.x + fgx), gy = G * (r.y + fgy), gz = G * (r.z + fgz);
                    double ph = G * (r.w + (fc - lin));
                    if (eps > 0.0) {  // take out the self pair's potential term (see eval_leaves1)
                        const double is = FP32C ? (double)__builtin_amdgcn_rsqf((float)e2) : rsq_nr1(e2);
                        ph += G * (m[q] * is);
                    }
                    if (accumulate) {
                        gxo[q] += gx;
                        gyo[q] += gy;
                        gzo[q] += gz;
                        if (deo) {  // thermokinetic form: the work of gravity on e = u + v^2/2
                            const double4 v = vel4[q];
                            deo[q] += fma(v.x, gx, fma(v.y, gy, v.z * gz));
                        }
                    } else {
                        gxo[q] = gx;
                        gyo[q] = gy;
                        gzo[q] = gz;
                    }
                    if (phi) pho[q] = ph;
                }
            }
        }
    }
}

void launch_fmm(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double G, double eps, double theta,
                int accumulate, int thermo) {
    if (dm.n <= 0) return;
    double* gx = accumulate ? d.ax : d.gx;
    double* gy = accumulate ? d.ay : d.gy;
    double* gz = accumulate ? d.az : d.gz;
    double* de = (accumulate && thermo) ? d.du : nullptr;
    const double th4 = 4.0 * (theta * theta);
    const double* ncell = &d.mom2[0].w;  // stride 4 doubles
    const int cg = std::min(2048, (dm.node_cap + 255) / 256);
    hipLaunchKernelGGL(k_fmm_cells, dim3(cg), dim3(256), 0, s, d.ctl, d.topo, d.range,
                       d.pos4, d.mom2);
    if (fp32c)
        hipLaunchKernelGGL(k_fmm<true>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.leaf_pre, d.pre_to_bfs, d.parent,
                           d.topo, d.range, d.mom0, ncell, d.pos4, d.m, G, eps, th4, accumulate, gx, gy, gz, d.phi,
                           d.vel4, de);
    else
        hipLaunchKernelGGL(k_fmm<false>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.leaf_pre, d.pre_to_bfs,
                           d.parent, d.topo, d.range, d.mom0, ncell, d.pos4, d.m, G, eps, th4, accumulate, gx, gy, gz,
                           d.phi, d.vel4, de);
}
