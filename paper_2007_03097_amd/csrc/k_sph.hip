// SPH pair sums (Sec. 2.2.1 of arXiv:2007.03097):
//   density (eq. (7)):  rho_a = sum_b m_b W(r_ab, h_ab), self included; ideal-gas EOS
//                       P = (gamma - 1) rho u, c = sqrt(gamma P / rho); h_next (eq. (9))
//   momentum (eq. (6)): dv_a/dt = -sum_b m_b ((P_a/rho_a^2 + P_b/rho_b^2) + Pi_ab) grad_a W_ab
//   energy (eq. (5)):   du_a/dt =  sum_b m_b (P_a/rho_a^2 + Pi_ab/2) v_ab . grad_a W_ab
//   or, thermokinetic (eq. (8)), e = u + v^2/2:
//                       de_a/dt = -sum_b m_b (P_a v_b/rho_a^2 + P_b v_a/rho_b^2
//                                             + (v_a + v_b)/2 Pi_ab) . grad_a W_ab
//   viscosity:          Pi_ab = (-alpha cbar mu + beta mu^2)/rhobar if v_ab . r_ab < 0,
//                       mu = h_ab v_ab . r_ab / (r^2 + eps h_ab^2)
// with the M4 cubic spline, W = w(q)/(pi h^3), grad_a W_ab = r_ab g(q)/(pi h^5), g = w'(q)/q.
//
// One 256-thread workgroup per target group, in an XCD-aware loop over the groups.  The group's
// source union (built with the lists) is staged in LDS in chunks; each of the group's n_g
// targets is served by PL = 256/n_g threads that take every PL-th entry of its list --
// entries are ascending union indices, so each thread walks its entries once across the
// chunks --
// and read the source records from LDS.  The partial sums of a target are added in a
// fixed order, so results are bitwise reproducible.  The pair sums are not a dense
// contraction (each target has its own irregular list), so they run on the vector ALUs,
// not on the matrix cores.
//
// FP32C: in the density pass positions enter as FP32 offsets from the group's first particle
// (each offset formed in FP64, then rounded), so a pair's difference is one FP32 subtraction
// of two nearby offsets; the force pass forms r_ab, v_ab and the support-edge margin
// (h_a + h_b)^2 - r^2 in FP64 and rounds them once (their rounding in FP32 would dominate the
// terms near the edge of the support and in smooth flows); everything
// else of the pair term is FP32, summed per thread with Kahan
// compensation (its error stays within about 2u times the sum of the terms' magnitudes,
// whatever their signs); the partial sums combine in FP64 and results are stored in FP64.
#include "common.h"

// rho, P, c given by the caller (caller order) -> key-ordered thermo records
__global__ void k_thermo_from_caller(int n, const u32* __restrict__ id, const double4* __restrict__ pos4,
                                     const double* __restrict__ rho, const double* __restrict__ P,
                                     const double* __restrict__ cs, double* drho, double* dP, double* dcs,
                                     double4* thr4, float4* thrf) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 i = id[q];
    const double r_ = rho[i], p_ = P[i], c_ = cs[i];
    const double pr2 = p_ / (r_ * r_);
    drho[q] = r_;
    dP[q] = p_;
    dcs[q] = c_;
    thr4[q] = make_double4(r_, pr2, c_, 0.0);
    thrf[q] = make_float4((float)r_, (float)pr2, (float)c_, (float)pos4[q].w);
}

void launch_thermo_from_caller(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* rho, const double* P,
                               const double* cs) {
    if (dm.n > 0)
        hipLaunchKernelGGL(k_thermo_from_caller, dim3((dm.n + 255) / 256), dim3(256), 0, s, dm.n, d.id, d.pos4, rho, P,
                           cs, d.rho, d.P, d.cs, d.thr4, d.thrf);
}

constexpr int PAIR_THREADS = 256;
constexpr int DENS_CHUNK = 512;
// Union sources staged per round of the force pass: FP64 records are 96 bytes, so 256 keep six
// workgroups per CU; the 48-byte FP32C records take 512, which covers most groups' union in one
// round (a wave runs each round as long as its busiest target, so fewer rounds waste fewer lanes).
constexpr int FORCE_CHUNK = 256;
constexpr int FORCE_CHUNK_F = 512;

// Density term of one pair: FP64, or FP32 on group-origin offsets with Kahan
// compensation.  One term is m_b w(r/h_ab) / h_ab^3 (1/pi applied at the end).
template <bool FP32C>
struct DensAcc;
template <>
struct DensAcc<false> {
    double s = 0.0;
    __device__ __forceinline__ void add(const double4 me, const double4 b, double mb) {
        const double dx = me.x - b.x, dy = me.y - b.y, dz = me.z - b.z;
        const double r = sqrt_nr(fma(dx, dx, fma(dy, dy, dz * dz)));
        const double ih = rcp_nr(0.5 * (me.w + b.w));
        s = fma(mb * m4_w(r * ih), ih * ih * ih, s);
    }
    __device__ __forceinline__ double value() const { return s; }
};
template <>
struct DensAcc<true> {
    Kahan k;
    // me, b: (x, y, z offsets from the group origin, h) in FP32
    __device__ __forceinline__ void add(const float4 me, const float4 b, float mb) {
        const float dx = me.x - b.x, dy = me.y - b.y, dz = me.z - b.z;
        const float r = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        const float ih = __builtin_amdgcn_rcpf(0.5f * (me.w + b.w));
        k.add(mb * m4_wf(r * ih) * (ih * ih * ih));
    }
    __device__ __forceinline__ double value() const { return k.value(); }
};

// FP32 offset record of a position from the group origin o: (x - o, y - o, z - o, h).
__device__ __forceinline__ float4 offset_rec(const double4 p, const double4 o) {
    return make_float4((float)(p.x - o.x), (float)(p.y - o.y), (float)(p.z - o.z), (float)p.w);
}


// An array of 32-byte records kept as two arrays of their 16-byte halves.  Read with 16-byte
// loads at random indices, records 32 bytes apart put the first half of every record in the
// same half of the LDS banks (a two-way conflict at least); at a 16-byte stride the halves of
// different records spread over all banks.
template <int N>
struct Split4 {
    double2 lo[N], hi[N];
    __device__ __forceinline__ void put(int i, const double4& v) {
        lo[i] = make_double2(v.x, v.y);
        hi[i] = make_double2(v.z, v.w);
    }
    __device__ __forceinline__ double4 get(int i) const {
        const double2 a = lo[i], b = hi[i];
        return make_double4(a.x, a.y, b.x, b.y);
    }
};

// Density sources staged in LDS: FP64 (x, y, z, h) and m, or FP32 offset records and m.
template <bool FP32C>
struct DensSrc;
template <>
struct DensSrc<false> {
    Split4<DENS_CHUNK> pos;
    double mass[DENS_CHUNK];
    using Rec = double4;
    using Mass = double;
    __device__ __forceinline__ void put(int i, const double4 p, double mb, const double4&) {
        pos.put(i, p);
        mass[i] = mb;
    }
    __device__ __forceinline__ double4 rec(int i) const { return pos.get(i); }
    __device__ __forceinline__ static double4 target(const double4 p, const double4&) { return p; }
};
template <>
struct DensSrc<true> {
    float4 pos[DENS_CHUNK];
    float mass[DENS_CHUNK];
    using Rec = float4;
    using Mass = float;
    __device__ __forceinline__ void put(int i, const double4 p, double mb, const double4& o) {
        pos[i] = offset_rec(p, o);
        mass[i] = (float)mb;
    }
    __device__ __forceinline__ float4 rec(int i) const { return pos[i]; }
    __device__ __forceinline__ static float4 target(const double4 p, const double4& o) { return offset_rec(p, o); }
};
static_assert(sizeof(DensSrc<true>) >= PAIR_THREADS * sizeof(double), "the reduction reuses the staging");

template <bool FP32C>
__global__ void __launch_bounds__(PAIR_THREADS) k_density(
    const DevCtl* __restrict__ ctl, const int4* __restrict__ group, int gsz, int cap, const u16* __restrict__ nbr,
    const int* __restrict__ nbr_cnt, const int* __restrict__ uni, const int* __restrict__ ucnt,
    const double4* __restrict__ pos4, const double4* __restrict__ vel4, const double* __restrict__ m,
    const double* __restrict__ u_eos, int kin, double gamma, double h_coeff, double* __restrict__ rho,
    double* __restrict__ P, double* __restrict__ cs, double* __restrict__ hnext, double4* __restrict__ thr4,
    float4* __restrict__ thrf) {
    __shared__ DensSrc<FP32C> S;
    const int tid = threadIdx.x;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
        const int4 g = group[gi];
        // PL = 256 / n_g threads per target, so a group with few targets still fills the
        // workgroup; thread tid serves target tid mod n_g (the last 256 mod n_g threads idle)
        const int PL = PAIR_THREADS / g.y;
        const int t = tid % g.y, phi = tid / g.y;
        const bool tv = phi < PL;
        const int q = g.x + t;
        const double4 org = pos4[g.x];  // group origin (FP32C offsets)
        const double4 mp = tv ? pos4[q] : make_double4(org.x, org.y, org.z, 1);
        const typename DensSrc<FP32C>::Rec me = DensSrc<FP32C>::target(mp, org);
        const int cnt = tv ? nbr_cnt[q] : 0;
        const u16* lst = nbr + (size_t)g.x * cap + t;
        const int* un = uni + (size_t)g.x * cap;
        const int nu = ucnt[gi];
        DensAcc<FP32C> acc;
        auto stage = [&](int c0, int cn) {  // union members c0 .. c0 + cn - 1 into LDS
            __syncthreads();
            for (int i = tid; i < cn; i += PAIR_THREADS) {
                const int b = un[c0 + i];
                S.put(i, pos4[b], m[b], org);
            }
            __syncthreads();
        };
        if constexpr (FP32C) {
            // The thread's entries k = phi, phi + PL, ... are read in batches of four, one batch
            // ahead of the batch being summed; every load goes to a register that is consumed only
            // after the next batch's loads are issued, and leaving a staged round keeps no loaded
            // value (the next round reloads from its slot), so no load is waited for early.  Slots
            // are clamped into the list (slot 0 of an empty list exists too); k < cnt decides.
            const int kmax = cnt > 0 ? cnt - 1 : 0;
            auto entry = [&](int kk) -> int { return lst[min(kk, kmax) * g.y]; };
            int k = phi;
            for (int c0 = 0; c0 < nu; c0 += DENS_CHUNK) {
                const int cn = nu - c0 < DENS_CHUNK ? nu - c0 : DENS_CHUNK;
                stage(c0, cn);
                const int ce = c0 + cn;
                auto take = [&](int r) {  // sums entry r if it is in the list and in this round
                    if (!(k < cnt && r < ce)) return false;
                    acc.add(me, S.rec(r - c0), S.mass[r - c0]);
                    k += PL;
                    return true;
                };
                int a0 = entry(k), a1 = entry(k + PL), a2 = entry(k + 2 * PL), a3 = entry(k + 3 * PL);
                while (true) {
                    const int b0 = entry(k + 4 * PL), b1 = entry(k + 5 * PL), b2 = entry(k + 6 * PL),
                              b3 = entry(k + 7 * PL);
                    if (!take(a0) || !take(a1) || !take(a2) || !take(a3)) break;
                    a0 = entry(k + 4 * PL);
                    a1 = entry(k + 5 * PL);
                    a2 = entry(k + 6 * PL);
                    a3 = entry(k + 7 * PL);
                    if (!take(b0) || !take(b1) || !take(b2) || !take(b3)) break;
                }
            }
        } else {  // the longer FP64 term hides a four-deep rotation's waits (batches measured slower)
            int k = phi;
            int e = k < cnt ? lst[k * g.y] : INT_MAX;
            int e1 = k + PL < cnt ? lst[(k + PL) * g.y] : INT_MAX;
            int e2 = k + 2 * PL < cnt ? lst[(k + 2 * PL) * g.y] : INT_MAX;
            int e3 = k + 3 * PL < cnt ? lst[(k + 3 * PL) * g.y] : INT_MAX;
            for (int c0 = 0; c0 < nu; c0 += DENS_CHUNK) {
                const int cn = nu - c0 < DENS_CHUNK ? nu - c0 : DENS_CHUNK;
                stage(c0, cn);
                const int ce = c0 + cn;
                while (e < ce) {
                    const int kn = k + 4 * PL;
                    const int en = kn < cnt ? lst[kn * g.y] : INT_MAX;
                    acc.add(me, S.rec(e - c0), S.mass[e - c0]);
                    k += PL;
                    e = e1;
                    e1 = e2;
                    e2 = e3;
                    e3 = en;
                }
            }
        }
        __syncthreads();
        double* red = reinterpret_cast<double*>(&S);
        red[tid] = acc.value();
        __syncthreads();
        if (tv && phi == 0) {
            double sum = red[t];
            for (int f = 1; f < PL; ++f) sum += red[t + g.y * f];
            const double r_ = sum * M_1_PI_D;
            double ue = u_eos[q];
            const double4 mpos = mp;
            if (kin) {  // u_eos holds the total energy e = u + v^2/2 (thermokinetic form)
                const double4 v = vel4[q];
                ue -= 0.5 * (v.x * v.x + v.y * v.y + v.z * v.z);
            }
            const double p_ = (gamma - 1.0) * r_ * ue;
            const double c_ = sqrt(gamma * p_ / r_);
            const double pr2 = p_ / (r_ * r_);
            rho[q] = r_;
            P[q] = p_;
            cs[q] = c_;
            hnext[q] = h_coeff * cbrt(m[q] / r_);
            thr4[q] = make_double4(r_, pr2, c_, ue);
            thrf[q] = make_float4((float)r_, (float)pr2, (float)c_, (float)mpos.w);
        }
    }
}

void launch_density(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double gamma, double h_coeff,
                    const double* u_eos, int kin) {
    if (dm.n <= 0) return;
    if (fp32c)
        hipLaunchKernelGGL(k_density<true>, dim3(dm.pair_grid), dim3(PAIR_THREADS), 0, s, d.ctl, d.group,
                           dm.group_size, dm.nbr_cap, d.nbr, d.nbr_cnt, d.uni, d.ucnt, d.pos4, d.vel4, d.m, u_eos,
                           kin, gamma, h_coeff, d.rho, d.P, d.cs, d.hnext, d.thr4, d.thrf);
    else
        hipLaunchKernelGGL(k_density<false>, dim3(dm.pair_grid), dim3(PAIR_THREADS), 0, s, d.ctl, d.group,
                           dm.group_size, dm.nbr_cap, d.nbr, d.nbr_cnt, d.uni, d.ucnt, d.pos4, d.vel4, d.m, u_eos,
                           kin, gamma, h_coeff, d.rho, d.P, d.cs, d.hnext, d.thr4, d.thrf);
}

// Source records in LDS for the force sums: FP64 (x, h), (v, m), (rho, P/rho^2, c), or
// FP32C (x, h) and (v, m) in FP64 and (rho, P/rho^2, c, h) in FP32.
template <bool FP32C>
struct ForceSrc;
template <>
struct ForceSrc<false> {
    Split4<FORCE_CHUNK> pos, vel, thr;
};
template <>
struct ForceSrc<true> {
    Split4<FORCE_CHUNK_F> pos, vel;  // x, y, z, h and predicted v, m in FP64: the pair's differences
    float4 thr[FORCE_CHUNK_F];       // and its support-edge margin are formed in FP64
};
static_assert(sizeof(ForceSrc<false>) >= 4 * PAIR_THREADS * sizeof(double), "the reduction reuses the staging");
static_assert(sizeof(ForceSrc<true>) >= 4 * PAIR_THREADS * sizeof(double), "the reduction reuses the staging");

template <bool FP32C, bool THERMO>
__global__ void __launch_bounds__(PAIR_THREADS) k_forces(
    const DevCtl* __restrict__ ctl, const int4* __restrict__ group, int gsz, int cap, const u16* __restrict__ nbr,
    const int* __restrict__ nbr_cnt, const int* __restrict__ uni, const int* __restrict__ ucnt,
    const double4* __restrict__ pos4, const double4* __restrict__ vel4, const double4* __restrict__ thr4,
    const float4* __restrict__ thrf, double alpha, double beta, double eps_av,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az, double* __restrict__ du) {
    __shared__ ForceSrc<FP32C> S;
    const int tid = threadIdx.x;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
        const int4 g = group[gi];
        // PL = 256 / n_g threads per target, so a group with few targets still fills the
        // workgroup; thread tid serves target tid mod n_g (the last 256 mod n_g threads idle)
        const int PL = PAIR_THREADS / g.y;
        const int t = tid % g.y, phi = tid / g.y;
        const bool tv = phi < PL;
        const int q = g.x + t;
        const double4 me = tv ? pos4[q] : make_double4(0, 0, 0, 1);
        const int cnt = tv ? nbr_cnt[q] : 0;
        const u16* lst = nbr + (size_t)g.x * cap + t;
        const int* un = uni + (size_t)g.x * cap;
        const int nu = ucnt[gi];
        int k = phi;
        double fx, fy, fz, fu;
        if constexpr (!FP32C) {
            int e = k < cnt ? lst[k * g.y] : INT_MAX;
            const double4 mv = tv ? vel4[q] : make_double4(0, 0, 0, 0);
            const double4 mt = tv ? thr4[q] : make_double4(1, 0, 0, 0);
            double sx = 0, sy = 0, sz = 0, su = 0;
            for (int c0 = 0; c0 < nu; c0 += FORCE_CHUNK) {
                const int cn = nu - c0 < FORCE_CHUNK ? nu - c0 : FORCE_CHUNK;
                __syncthreads();
                for (int i = tid; i < cn; i += PAIR_THREADS) {
                    const int b = un[c0 + i];
                    S.pos.put(i, pos4[b]);
                    S.vel.put(i, vel4[b]);
                    S.thr.put(i, thr4[b]);
                }
                __syncthreads();
                const int ce = c0 + cn;
                while (e < ce) {
                    const int kn = k + PL;
                    const int en = kn < cnt ? lst[kn * g.y] : INT_MAX;
                    const int j = e - c0;
                    const double4 sb = S.pos.get(j);
                    const double4 vb = S.vel.get(j);
                    const double4 tb = S.thr.get(j);
                    const double dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    double ir;
                    const double r = sqrt_rsq_nr(r2, ir);
                    const double hab = 0.5 * (me.w + sb.w);
                    const double ih = rcp_nr(hab);
                    const double ih2 = ih * ih;
                    const double qq = r * ih;
                    const double gw = m4_g(qq, hab * ir) * (ih2 * ih2 * ih) * M_1_PI_D;
                    const double wx = mv.x - vb.x, wy = mv.y - vb.y, wz = mv.z - vb.z;
                    const double vr = fma(wx, dx, fma(wy, dy, wz * dz));
                    double Pi = 0.0;
                    if (vr < 0.0) {  // one reciprocal of den * rhobar gives 1/den and 1/rhobar
                        const double den = fma(eps_av * hab, hab, r2);
                        const double rb = 0.5 * (mt.x + tb.x);
                        const double inv = rcp_nr(den * rb);
                        const double mu = hab * vr * (rb * inv);
                        Pi = fma(-alpha * 0.5 * (mt.z + tb.z), mu, beta * mu * mu) * (den * inv);
                    }
                    const double term = vb.w * ((mt.y + tb.y) + Pi) * gw;
                    sx = fma(-term, dx, sx);
                    sy = fma(-term, dy, sy);
                    sz = fma(-term, dz, sz);
                    if (THERMO) {  // eq. (8): P_a v_b/rho_a^2 + P_b v_a/rho_b^2 + (v_a + v_b)/2 Pi
                        const double var = fma(mv.x, dx, fma(mv.y, dy, mv.z * dz));
                        const double vbr = fma(vb.x, dx, fma(vb.y, dy, vb.z * dz));
                        su = fma(-vb.w * gw, fma(mt.y, vbr, fma(tb.y, var, 0.5 * Pi * (var + vbr))), su);
                    } else {
                        su = fma(vb.w * fma(0.5, Pi, mt.y) * gw, vr, su);
                    }
                    k = kn;
                    e = en;
                }
            }
            fx = sx; fy = sy; fz = sz; fu = su;
        } else {
            const double4 mv = tv ? vel4[q] : make_double4(0, 0, 0, 0);
            const float4 mt = tv ? thrf[q] : make_float4(1, 0, 0, 1);
            const float alf = (float)alpha, bef = (float)beta, epf = (float)eps_av;
            const float ipi = (float)M_1_PI_D;
            Kahan sx, sy, sz, su;
            // entries read in batches of four, one batch ahead (as in the FP32C density pass)
            const int kmax = cnt > 0 ? cnt - 1 : 0;
            auto entry = [&](int kk) -> int { return lst[min(kk, kmax) * g.y]; };
            for (int c0 = 0; c0 < nu; c0 += FORCE_CHUNK_F) {
                const int cn = nu - c0 < FORCE_CHUNK_F ? nu - c0 : FORCE_CHUNK_F;
                __syncthreads();
                for (int i = tid; i < cn; i += PAIR_THREADS) {
                    const int b = un[c0 + i];
                    S.pos.put(i, pos4[b]);
                    S.vel.put(i, vel4[b]);
                    S.thr[i] = thrf[b];
                }
                __syncthreads();
                const int ce = c0 + cn;
                auto take = [&](int ent) {
                    if (!(k < cnt && ent < ce)) return false;
                    const int j = ent - c0;
                    const double4 sb = S.pos.get(j);
                    const double4 vb = S.vel.get(j);
                    const float4 tb = S.thr[j];
                    // the pair's separation, relative velocity and margin to the support edge
                    // in FP64, rounded once to FP32: D = (h_a + h_b)^2 - r^2 has no
                    // cancellation, so 2 - q = D/((T + r) h_ab) keeps FP32 relative accuracy as
                    // q -> 2 (2 - q formed from an FP32 q loses digits there), and r_ab, v_ab
                    // keep it however large the positions and velocities are against their
                    // differences; the rest of the pair term is FP32
                    const double ex = me.x - sb.x, ey = me.y - sb.y, ez = me.z - sb.z;
                    const double r2d = fma(ex, ex, fma(ey, ey, ez * ez));
                    const double Td = me.w + sb.w;
                    const float Dm = (float)fma(Td, Td, -r2d);
                    const float dx = (float)ex, dy = (float)ey, dz = (float)ez;
                    const float r2 = (float)r2d;
                    const float r = __builtin_amdgcn_sqrtf(r2);
                    const float T = (float)Td;
                    const float hab = 0.5f * T;
                    const float ih = __builtin_amdgcn_rcpf(hab);
                    const float ih2 = ih * ih;
                    const float qq = r * ih;
                    const float tq = Dm * __builtin_amdgcn_rcpf((T + r) * hab);
                    const float gq = qq < 1.0f ? fmaf(2.25f, qq, -3.0f) : -0.75f * (tq * tq) * __builtin_amdgcn_rcpf(qq);
                    const float gw = gq * (ih2 * ih2 * ih) * ipi;
                    const float wx = (float)(mv.x - vb.x), wy = (float)(mv.y - vb.y), wz = (float)(mv.z - vb.z);
                    const float vr = fmaf(wx, dx, fmaf(wy, dy, wz * dz));
                    float Pi = 0.0f;
                    if (vr < 0.0f) {
                        const float mu = hab * vr * __builtin_amdgcn_rcpf(fmaf(epf * hab, hab, r2));
                        Pi = fmaf(-alf * 0.5f * (mt.z + tb.z), mu, bef * mu * mu) *
                             __builtin_amdgcn_rcpf(0.5f * (mt.x + tb.x));
                    }
                    const float mb = (float)vb.w;
                    const float term = mb * ((mt.y + tb.y) + Pi) * gw;
                    sx.add(-term * dx);
                    sy.add(-term * dy);
                    sz.add(-term * dz);
                    if (THERMO) {  // eq. (8) takes the absolute velocities
                        const float var = fmaf((float)mv.x, dx, fmaf((float)mv.y, dy, (float)mv.z * dz));
                        const float vbr = fmaf((float)vb.x, dx, fmaf((float)vb.y, dy, (float)vb.z * dz));
                        su.add(-mb * gw * fmaf(mt.y, vbr, fmaf(tb.y, var, 0.5f * Pi * (var + vbr))));
                    } else {
                        su.add(mb * fmaf(0.5f, Pi, mt.y) * gw * vr);
                    }
                    k += PL;
                    return true;
                };
                int a0 = entry(k), a1 = entry(k + PL), a2 = entry(k + 2 * PL), a3 = entry(k + 3 * PL);
                while (true) {
                    const int b0 = entry(k + 4 * PL), b1 = entry(k + 5 * PL), b2 = entry(k + 6 * PL),
                              b3 = entry(k + 7 * PL);
                    if (!take(a0) || !take(a1) || !take(a2) || !take(a3)) break;
                    a0 = entry(k + 4 * PL);
                    a1 = entry(k + 5 * PL);
                    a2 = entry(k + 6 * PL);
                    a3 = entry(k + 7 * PL);
                    if (!take(b0) || !take(b1) || !take(b2) || !take(b3)) break;
                }
            }
            fx = sx.value(); fy = sy.value(); fz = sz.value(); fu = su.value();
        }
        __syncthreads();
        double* red = reinterpret_cast<double*>(&S);  // 4 x 256 doubles
        red[tid] = fx;
        red[PAIR_THREADS + tid] = fy;
        red[2 * PAIR_THREADS + tid] = fz;
        red[3 * PAIR_THREADS + tid] = fu;
        __syncthreads();
        if (tv && phi == 0) {
            double s0 = red[t], s1 = red[PAIR_THREADS + t], s2 = red[2 * PAIR_THREADS + t], s3 = red[3 * PAIR_THREADS + t];
            for (int f = 1; f < PL; ++f) {
                const int i = t + g.y * f;
                s0 += red[i];
                s1 += red[PAIR_THREADS + i];
                s2 += red[2 * PAIR_THREADS + i];
                s3 += red[3 * PAIR_THREADS + i];
            }
            ax[q] = s0;
            ay[q] = s1;
            az[q] = s2;
            du[q] = s3;
        }
    }
}

void launch_forces(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double alpha, double beta,
                   double eps_av, int thermo) {
    if (dm.n <= 0) return;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(dm.pair_grid), dim3(PAIR_THREADS), 0, s, d.ctl, d.group, dm.group_size,
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.uni, d.ucnt, d.pos4, d.vel4, d.thr4, d.thrf, alpha,
                           beta, eps_av, d.ax, d.ay, d.az, d.du);
    };
    if (fp32c) {
        if (thermo) go(k_forces<true, true>);
        else go(k_forces<true, false>);
    } else {
        if (thermo) go(k_forces<false, true>);
        else go(k_forces<false, false>);
    }
}
