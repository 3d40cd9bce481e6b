// Octree self-gravity (Sec. 2.2.2 of arXiv:2007.03097, eq. (10), with Plummer softening
// and quadrupole moments).
//
// One wavefront per target group.  The wide walk tests up to 64 nodes at once against the
// group's box: a cell B of side s_B is accepted for the whole group when its particle box
// does not touch the group box and s_B < theta d, d being the distance from B's centre of
// mass to the group box (theta = 0 opens everything: the exact direct sum).  Accepted
// cells act through the second-order expansion of the softened potential about their
// centre of mass (monopole + quadrupole; the dipole vanishes there):
//   phi += -G [M/s + (3/2) R.I.R/s^5 - (1/2) tr(I)/s^3]
//   g   +=  G [-M R/s^3 + 3 I.R/s^5 - (15/2) (R.I.R) R/s^7 + (3/2) tr(I) R/s^5]
// with R = r_a - R_B, s^2 = |R|^2 + eps^2, I = sum m y y^T about R_B.  Unaccepted leaves
// contribute softened particle sums with the target itself skipped.  Cell and leaf lists
// live in LDS and are evaluated whenever they fill, so the walk needs no global scratch;
// the evaluation stages cell moments and leaf particles through LDS 64 at a time.
#include "common.h"

constexpr int GW_STACK = 512;
constexpr int GW_CELLS = 512;
constexpr int GW_LEAVES = 256;

struct GravAcc {
    double gx = 0, gy = 0, gz = 0, ph = 0;
};

// LDS staging of one evaluation: cell moments in the cell phase, particles in the leaf phase.
struct GravStage {
    union {
        struct {
            double4 c0[64], c1[64], c2[64];  // (M, com), (Ixx, Iyy, Izz, tr I), (Ixy, Ixz, Iyz, -)
        } cell;
        struct {
            double4 pm[64];  // (x, y, z, m)
            int src[64];     // particle index (self test without softening)
        } part;
    };
    int loff[GW_LEAVES + 1];  // particle offsets of the staged leaves
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

// Accepted cells (monopole + quadrupole) and unaccepted leaves (softened particle sums,
// self skipped) for target `me` (index q).  Cells are staged 64 at a time (one lane loads
// one cell); the leaves' particles are concatenated and staged 64 at a time, so every
// staging round is one load per lane.  Lane (t, phi) takes every P_-th staged item.
// Accepted cells (monopole + quadrupole) and unaccepted leaves (softened particle sums,
// self excluded) for target `me` (index q).  Cells are staged 64 at a time (one lane loads
// one cell); the leaves' particles are concatenated and staged 64 at a time, so every
// staging round is one load per lane.  Lane (t, phi) takes every P_-th staged item.
// FP32C: the terms of one staged tile are summed in FP32, and the tile sums enter Kahan-
// compensated FP32 accumulators.  With softening the self pair is evaluated like any
// other (it adds no force) and its potential term -m_q/eps is taken out at the end.
template <bool FP32C>
__device__ void eval_lists(int ncell, int nleaf, const int* cells, int* leaves, GravStage& S,
                           const int4* __restrict__ topo, const double4* __restrict__ mom0,
                           const double4* __restrict__ mom1, const double4* __restrict__ mom2,
                           const double4* __restrict__ pos4, const double* __restrict__ m, const double4 me, int q,
                           bool tv, int phi, int P_, double G, double eps, GravAcc& acc) {
    const int lane = lane_id();
    const double e2 = eps * eps;
    double cgx = 0, cgy = 0, cgz = 0, cph = 0;
    KahanF kx, ky, kz, kp;
    // ---- cells
    for (int k0 = 0; k0 < ncell; k0 += 64) {
        __syncthreads();
        if (k0 + lane < ncell) {
            const int c = cells[k0 + lane];
            S.cell.c0[lane] = mom0[c];
            S.cell.c1[lane] = mom1[c];
            S.cell.c2[lane] = mom2[c];
        }
        __syncthreads();
        const int cn = ncell - k0 < 64 ? ncell - k0 : 64;
        if (!tv) continue;
        float tx = 0.0f, ty = 0.0f, tz = 0.0f, tph = 0.0f;
        for (int k = phi; k < cn; k += P_) {
            const double4 a = S.cell.c0[k], b = S.cell.c1[k], d = S.cell.c2[k];
            if (!FP32C) {
                const double Rx = me.x - a.y, Ry = me.y - a.z, Rz = me.z - a.w;
                const double IRx = fma(b.x, Rx, fma(d.x, Ry, d.y * Rz));
                const double IRy = fma(d.x, Rx, fma(b.y, Ry, d.z * Rz));
                const double IRz = fma(d.y, Rx, fma(d.z, Ry, b.z * Rz));
                const double RIR = fma(Rx, IRx, fma(Ry, IRy, Rz * IRz));
                const double s2 = fma(Rx, Rx, fma(Ry, Ry, fma(Rz, Rz, e2)));
                const double i1 = rsq_nr(s2);
                const double i2 = i1 * i1, i3 = i1 * i2, i5 = i3 * i2, i7 = i5 * i2;
                const double cR = -a.x * i3 + 1.5 * b.w * i5 - 7.5 * RIR * i7;
                cgx = fma(cR, Rx, fma(3.0 * i5, IRx, cgx));
                cgy = fma(cR, Ry, fma(3.0 * i5, IRy, cgy));
                cgz = fma(cR, Rz, fma(3.0 * i5, IRz, cgz));
                cph -= a.x * i1 + 1.5 * RIR * i5 - 0.5 * b.w * i3;
            } else {
                const float Rx = (float)(me.x - a.y), Ry = (float)(me.y - a.z), Rz = (float)(me.z - a.w);
                const float bx = (float)b.x, by = (float)b.y, bz = (float)b.z, tr = (float)b.w;
                const float dxy = (float)d.x, dxz = (float)d.y, dyz = (float)d.z, M = (float)a.x;
                const float IRx = fmaf(bx, Rx, fmaf(dxy, Ry, dxz * Rz));
                const float IRy = fmaf(dxy, Rx, fmaf(by, Ry, dyz * Rz));
                const float IRz = fmaf(dxz, Rx, fmaf(dyz, Ry, bz * Rz));
                const float RIR = fmaf(Rx, IRx, fmaf(Ry, IRy, Rz * IRz));
                const float s2 = fmaf(Rx, Rx, fmaf(Ry, Ry, fmaf(Rz, Rz, (float)e2)));
                const float i1 = __builtin_amdgcn_rsqf(s2);
                const float i2 = i1 * i1, i3 = i1 * i2, i5 = i3 * i2, i7 = i5 * i2;
                const float cR = -M * i3 + 1.5f * tr * i5 - 7.5f * RIR * i7;
                tx = fmaf(cR, Rx, fmaf(3.0f * i5, IRx, tx));
                ty = fmaf(cR, Ry, fmaf(3.0f * i5, IRy, ty));
                tz = fmaf(cR, Rz, fmaf(3.0f * i5, IRz, tz));
                tph -= M * i1 + 1.5f * RIR * i5 - 0.5f * tr * i3;
            }
        }
        if (FP32C) {
            kx.add(tx); ky.add(ty); kz.add(tz); kp.add(tph);
        }
    }
    // ---- leaves: offsets of their particles, then the particles 64 at a time
    int carry = 0;
    for (int j0 = 0; j0 < nleaf; j0 += 64) {
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
            S.loff[j] = carry + incl - c;
        }
        carry += __shfl(incl, 63, 64);
    }
    __syncthreads();
    const int total = carry;
    const bool soft = e2 > 0.0;
    for (int p0 = 0; p0 < total; p0 += 64) {
        const int p = p0 + lane;
        __syncthreads();
        if (p < total) {
            int a = 0, b = nleaf - 1;
            while (a < b) {  // largest j with loff[j] <= p
                const int mid = (a + b + 1) >> 1;
                if (S.loff[mid] <= p) a = mid;
                else b = mid - 1;
            }
            const int src = leaves[a] + (p - S.loff[a]);
            const double4 ps = pos4[src];
            S.part.pm[lane] = make_double4(ps.x, ps.y, ps.z, m[src]);
            S.part.src[lane] = src;
        }
        __syncthreads();
        const int tn = total - p0 < 64 ? total - p0 : 64;
        if (!tv) continue;
        float tx = 0.0f, ty = 0.0f, tz = 0.0f, tph = 0.0f;
        for (int j = phi; j < tn; j += P_) {
            const double4 sb = S.part.pm[j];
            if (!soft && S.part.src[j] == q) continue;
            if (!FP32C) {
                const double dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
                const double s2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, e2)));
                const double i1 = rsq_nr(s2);
                const double mi3 = sb.w * i1 * i1 * i1;
                cgx = fma(-mi3, dx, cgx);
                cgy = fma(-mi3, dy, cgy);
                cgz = fma(-mi3, dz, cgz);
                cph = fma(-sb.w, i1, cph);
            } else {
                const float dx = (float)(me.x - sb.x), dy = (float)(me.y - sb.y), dz = (float)(me.z - sb.z);
                const float s2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, (float)e2)));
                const float i1 = __builtin_amdgcn_rsqf(s2);
                const float mb = (float)sb.w;
                const float mi3 = mb * i1 * i1 * i1;
                tx = fmaf(-mi3, dx, tx);
                ty = fmaf(-mi3, dy, ty);
                tz = fmaf(-mi3, dz, tz);
                tph = fmaf(-mb, i1, tph);
            }
        }
        if (FP32C) {
            kx.add(tx); ky.add(ty); kz.add(tz); kp.add(tph);
        }
    }
    if (FP32C) {
        cgx = kx.value();
        cgy = ky.value();
        cgz = kz.value();
        cph = kp.value();
    }
    acc.gx += G * cgx;
    acc.gy += G * cgy;
    acc.gz += G * cgz;
    acc.ph += G * cph;
}

template <bool FP32C>
__global__ void __launch_bounds__(64) k_gravity(DevCtl* ctl, const int4* __restrict__ group, int gsz,
                                                const int4* __restrict__ topo, const double4* __restrict__ nbox_lo,
                                                const double4* __restrict__ nbox_hi, const double4* __restrict__ mom0,
                                                const double4* __restrict__ mom1, const double4* __restrict__ mom2,
                                                const double4* __restrict__ pos4, const double* __restrict__ m,
                                                double G, double eps, double theta, int accumulate,
                                                double* __restrict__ gxo, double* __restrict__ gyo,
                                                double* __restrict__ gzo, double* __restrict__ pho) {
    __shared__ int stack[GW_STACK];
    __shared__ int cells[GW_CELLS];
    __shared__ int leaves[GW_LEAVES];
    __shared__ GravStage S;
    const int lane = lane_id();
    const int t = lane & (gsz - 1), phi = lane / gsz, P_ = 64 / gsz;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
    const int4 g = group[gi];
    const bool tv = t < g.y;
    const int q = g.x + t;
    const double4 me = tv ? pos4[q] : make_double4(0, 0, 0, 0);
    double lo[3], hi[3];
    lo[0] = wave_min(tv ? me.x : INFINITY); hi[0] = wave_max(tv ? me.x : -INFINITY);
    lo[1] = wave_min(tv ? me.y : INFINITY); hi[1] = wave_max(tv ? me.y : -INFINITY);
    lo[2] = wave_min(tv ? me.z : INFINITY); hi[2] = wave_max(tv ? me.z : -INFINITY);
    const double th2 = theta * theta;
    const u64 lt = lanemask_lt();
    GravAcc acc;
    const int root = g.z < 0 ? 0 : ctl->level_off[3] + g.z;
    __syncthreads();
    if (lane == 0) stack[0] = root;
    int sp = 1, nc = 0, nl = 0, iters = 0;
    __syncthreads();
    while (sp > 0) {
        if (++iters > (1 << 22)) {  // bounded: every wave leaves the loop
            if (lane == 0) set_err(ctl, ERR_GRAV_LIST);
            break;
        }
        if (nc + 64 > GW_CELLS || nl + 64 > GW_LEAVES) {
            eval_lists<FP32C>(nc, nl, cells, leaves, S, topo, mom0, mom1, mom2, pos4, m, me, q, tv, phi, P_,
                              G, eps, acc);
            nc = nl = 0;
            __syncthreads();
        }
        int k = sp < 64 ? sp : 64;
        const int room = (GW_STACK - sp) / 8;
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
            const bool apart = a.x > hi[0] || b.x < lo[0] || a.y > hi[1] || b.y < lo[1] || a.z > hi[2] || b.z < lo[2];
            const double side = b.w;
            if (apart && side * side < th2 * d2) kind = 1;
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
    eval_lists<FP32C>(nc, nl, cells, leaves, S, topo, mom0, mom1, mom2, pos4, m, me, q, tv, phi, P_, G, eps,
                      acc);
    acc.gx = lanes_sum_d(acc.gx, gsz);
    acc.gy = lanes_sum_d(acc.gy, gsz);
    acc.gz = lanes_sum_d(acc.gz, gsz);
    acc.ph = lanes_sum_d(acc.ph, gsz);
    if (tv && phi == 0) {
        if (eps > 0.0) {  // take out the self pair's potential term (see eval_lists)
            const double e2 = eps * eps;
            const double is = FP32C ? (double)__builtin_amdgcn_rsqf((float)e2) : rsq_nr(e2);
            acc.ph += G * (m[q] * is);
        }
        if (accumulate) {
            gxo[q] += acc.gx;
            gyo[q] += acc.gy;
            gzo[q] += acc.gz;
        } else {
            gxo[q] = acc.gx;
            gyo[q] = acc.gy;
            gzo[q] = acc.gz;
        }
        if (pho) pho[q] = acc.ph;
    }
    }
}

void launch_gravity(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double G, double eps, double theta,
                    int accumulate) {
    if (dm.n <= 0) return;
    double* gx = accumulate ? d.ax : d.gx;
    double* gy = accumulate ? d.ay : d.gy;
    double* gz = accumulate ? d.az : d.gz;
    if (fp32c)
        hipLaunchKernelGGL(k_gravity<true>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size, d.topo,
                           d.nbox_lo, d.nbox_hi, d.mom0, d.mom1, d.mom2, d.pos4, d.m, G, eps, theta, accumulate, gx, gy,
                           gz, d.phi);
    else
        hipLaunchKernelGGL(k_gravity<false>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size, d.topo,
                           d.nbox_lo, d.nbox_hi, d.mom0, d.mom1, d.mom2, d.pos4, d.m, G, eps, theta, accumulate, gx, gy,
                           gz, d.phi);
}
