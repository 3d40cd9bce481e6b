// SPH pair sums (Sec. 2.2.1 of arXiv:2007.03097).
//
//   density (eq. (7)):  rho_a = sum_b m_b W(r_ab, h_ab),  h_ab = (h_a + h_b)/2, self included
//   EOS:                P = (gamma - 1) rho u,  c = sqrt(gamma P / rho)
//   eq. (9):            h_next = h_coeff (m / rho)^(1/3)
//   momentum (eq. (6)): dv_a/dt = -sum_b m_b ((P_a/rho_a^2 + P_b/rho_b^2) + Pi_ab) grad_a W_ab
//   energy (eq. (5)):   du_a/dt =  sum_b m_b (P_a/rho_a^2 + Pi_ab/2) v_ab . grad_a W_ab
//   viscosity:          Pi_ab = (-alpha cbar mu + beta mu^2)/rhobar if v_ab . r_ab < 0,
//                       mu = h_ab v_ab . r_ab / (r^2 + eps h_ab^2)
// with the M4 cubic spline W = w(q)/(pi h^3), grad_a W_ab = r_ab g(q)/(pi h^5), g = w'(q)/q.
//
// One wavefront per group of group_size targets (four consecutive groups per workgroup, so
// their neighbour gathers share one L1); target t is served by 64/group_size lanes that take
// every (64/group_size)-th entry of its neighbour list, then combine in a fixed butterfly
// order, so results are bitwise reproducible.  The pair sums are not a
// dense contraction (each target has its own irregular list), so they run on the vector
// ALUs, not on the matrix cores.
//
// FP32C: the position difference is formed in FP64 and rounded to FP32; everything else
// of the pair term is FP32, summed per lane with Kahan (density) or Neumaier (momentum,
// energy) compensation; lanes combine in FP64 and results are stored in FP64.
#include "common.h"

__device__ __forceinline__ double m4_w(double q) {
    if (q < 1.0) return fma(q * q, fma(0.75, q, -1.5), 1.0);
    if (q < 2.0) {
        const double t = 2.0 - q;
        return 0.25 * t * t * t;
    }
    return 0.0;
}
__device__ __forceinline__ double m4_g(double q) {
    if (q < 1.0) return fma(2.25, q, -3.0);
    if (q < 2.0) {
        const double t = 2.0 - q;
        return -0.75 * t * t / q;
    }
    return 0.0;
}
__device__ __forceinline__ float m4_wf(float q) {
    if (q < 1.0f) return fmaf(q * q, fmaf(0.75f, q, -1.5f), 1.0f);
    if (q < 2.0f) {
        const float t = 2.0f - q;
        return 0.25f * t * t * t;
    }
    return 0.0f;
}
__device__ __forceinline__ float m4_gf(float q, float inv_q) {
    if (q < 1.0f) return fmaf(2.25f, q, -3.0f);
    if (q < 2.0f) {
        const float t = 2.0f - q;
        return -0.75f * t * t * inv_q;
    }
    return 0.0f;
}


// Kahan / Neumaier accumulators (explicit operation order; the library is built without
// floating-point contraction, so these are not fused).
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
struct Neumaier {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x) {
        const float t = s + x;
        c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s + (double)c; }
};

// ---------------------------------------------------------------------------------------
template <bool FP32C>
__global__ void __launch_bounds__(256) k_density(const DevCtl* __restrict__ ctl, const int4* __restrict__ group,
                                                int gsz, int cap,
                                                const int* __restrict__ nbr, const int* __restrict__ nbr_cnt,
                                                const double4* __restrict__ pos4, const double* __restrict__ m,
                                                const double* __restrict__ u_eos, double gamma, double h_coeff,
                                                double* __restrict__ rho, double* __restrict__ P,
                                                double* __restrict__ cs, double* __restrict__ hnext,
                                                double4* __restrict__ thr4, float4* __restrict__ thrf) {
    const int lane = lane_id();
    const int t = lane & (gsz - 1), phi = lane / gsz, P_ = 64 / gsz;
    const int ng = ctl->n_groups;
    int g0, g1, gstep;
    group_range((ng + 3) >> 2, g0, g1, gstep);   // four consecutive groups per workgroup share L1
    for (int gq = g0; gq < g1; gq += gstep) {
    const int gi = 4 * gq + (int)(threadIdx.x >> 6);
    if (gi >= ng) continue;
    const int4 g = group[gi];
    const bool tv = t < g.y;
    const int q = g.x + t;
    const double4 me = tv ? pos4[q] : make_double4(0, 0, 0, 1);
    const int cnt = tv ? nbr_cnt[q] : 0;
    const int* lst = nbr + (size_t)g.x * cap + t;
    double acc;
    if (!FP32C) {
        double s = 0.0;
        for (int k = phi; k < cnt; k += P_) {
            const int b = lst[k * g.y];
            const double4 sb = pos4[b];
            const double dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
            const double r = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
            const double ih = 1.0 / (0.5 * (me.w + sb.w));
            s = fma(m[b] * m4_w(r * ih), ih * ih * ih, s);
        }
        acc = s;
    } else {
        Kahan s;
        const float hf = (float)me.w;
        for (int k = phi; k < cnt; k += P_) {
            const int b = lst[k * g.y];
            const double4 sb = pos4[b];
            const float dx = (float)(me.x - sb.x), dy = (float)(me.y - sb.y), dz = (float)(me.z - sb.z);
            const float r = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            const float ih = __builtin_amdgcn_rcpf(0.5f * (hf + (float)sb.w));
            s.add((float)m[b] * m4_wf(r * ih) * (ih * ih * ih));
        }
        acc = s.value();
    }
    acc = lanes_sum_d(acc, gsz);
    if (tv && phi == 0) {
        const double r_ = acc * M_1_PI_D;
        const double ue = u_eos[q];
        const double p_ = (gamma - 1.0) * r_ * ue;
        const double c_ = sqrt(gamma * p_ / r_);
        const double pr2 = p_ / (r_ * r_);
        rho[q] = r_;
        P[q] = p_;
        cs[q] = c_;
        hnext[q] = h_coeff * cbrt(m[q] / r_);
        thr4[q] = make_double4(r_, pr2, c_, ue);
        thrf[q] = make_float4((float)r_, (float)pr2, (float)c_, (float)me.w);
    }
    }
}

void launch_density(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double gamma, double h_coeff,
                    const double* u_eos) {
    if (dm.n <= 0) return;
    if (fp32c)
        hipLaunchKernelGGL(k_density<true>, dim3(dm.group_grid / 4 > 8 ? (dm.group_grid / 4) & ~7 : 8), dim3(256), 0, s, d.ctl, d.group, dm.group_size, dm.nbr_cap,
                           d.nbr, d.nbr_cnt, d.pos4, d.m, u_eos, gamma, h_coeff, d.rho, d.P, d.cs, d.hnext, d.thr4,
                           d.thrf);
    else
        hipLaunchKernelGGL(k_density<false>, dim3(dm.group_grid / 4 > 8 ? (dm.group_grid / 4) & ~7 : 8), dim3(256), 0, s, d.ctl, d.group, dm.group_size, dm.nbr_cap,
                           d.nbr, d.nbr_cnt, d.pos4, d.m, u_eos, gamma, h_coeff, d.rho, d.P, d.cs, d.hnext, d.thr4,
                           d.thrf);
}

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

// ---------------------------------------------------------------------------------------
template <bool FP32C>
__global__ void __launch_bounds__(256) k_forces(const DevCtl* __restrict__ ctl, const int4* __restrict__ group,
                                               int gsz, int cap,
                                               const int* __restrict__ nbr, const int* __restrict__ nbr_cnt,
                                               const double4* __restrict__ pos4, const double4* __restrict__ vel4,
                                               const double4* __restrict__ thr4, const float4* __restrict__ velf,
                                               const float4* __restrict__ thrf, double alpha, double beta,
                                               double eps_av, double* __restrict__ ax, double* __restrict__ ay,
                                               double* __restrict__ az, double* __restrict__ du) {
    const int lane = lane_id();
    const int t = lane & (gsz - 1), phi = lane / gsz, P_ = 64 / gsz;
    const int ng = ctl->n_groups;
    int g0, g1, gstep;
    group_range((ng + 3) >> 2, g0, g1, gstep);   // four consecutive groups per workgroup share L1
    for (int gq = g0; gq < g1; gq += gstep) {
    const int gi = 4 * gq + (int)(threadIdx.x >> 6);
    if (gi >= ng) continue;
    const int4 g = group[gi];
    const bool tv = t < g.y;
    const int q = g.x + t;
    const double4 me = tv ? pos4[q] : make_double4(0, 0, 0, 1);
    const int cnt = tv ? nbr_cnt[q] : 0;
    const int* lst = nbr + (size_t)g.x * cap + t;
    double fx, fy, fz, fu;
    if (!FP32C) {
        const double4 mv = tv ? vel4[q] : make_double4(0, 0, 0, 0);
        const double4 mt = tv ? thr4[q] : make_double4(1, 0, 0, 0);
        double sx = 0, sy = 0, sz = 0, su = 0;
        for (int k = phi; k < cnt; k += P_) {
            const int b = lst[k * g.y];
            const double4 sb = pos4[b];
            const double4 vb = vel4[b];
            const double4 tb = thr4[b];
            const double dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double r = sqrt(r2);
            const double hab = 0.5 * (me.w + sb.w);
            const double ih = 1.0 / hab;
            const double ih2 = ih * ih;
            const double gw = m4_g(r * ih) * (ih2 * ih2 * ih) * M_1_PI_D;
            const double wx = mv.x - vb.x, wy = mv.y - vb.y, wz = mv.z - vb.z;
            const double vr = fma(wx, dx, fma(wy, dy, wz * dz));
            double Pi = 0.0;
            if (vr < 0.0) {
                const double mu = hab * vr / fma(eps_av * hab, hab, r2);
                Pi = fma(-alpha * 0.5 * (mt.z + tb.z), mu, beta * mu * mu) / (0.5 * (mt.x + tb.x));
            }
            const double term = vb.w * ((mt.y + tb.y) + Pi) * gw;
            sx = fma(-term, dx, sx);
            sy = fma(-term, dy, sy);
            sz = fma(-term, dz, sz);
            su = fma(vb.w * fma(0.5, Pi, mt.y) * gw, vr, su);
        }
        fx = sx; fy = sy; fz = sz; fu = su;
    } else {
        const float4 mv = tv ? velf[q] : make_float4(0, 0, 0, 0);
        const float4 mt = tv ? thrf[q] : make_float4(1, 0, 0, 1);
        const float alf = (float)alpha, bef = (float)beta, epf = (float)eps_av;
        const float ipi = (float)M_1_PI_D;
        Neumaier sx, sy, sz, su;
        for (int k = phi; k < cnt; k += P_) {
            const int b = lst[k * g.y];
            const double4 sb = pos4[b];
            const float4 vb = velf[b];
            const float4 tb = thrf[b];
            const float dx = (float)(me.x - sb.x), dy = (float)(me.y - sb.y), dz = (float)(me.z - sb.z);
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float r = __builtin_amdgcn_sqrtf(r2);
            const float hab = 0.5f * (mt.w + tb.w);
            const float ih = __builtin_amdgcn_rcpf(hab);
            const float ih2 = ih * ih;
            const float qq = r * ih;
            const float gw = m4_gf(qq, __builtin_amdgcn_rcpf(qq)) * (ih2 * ih2 * ih) * ipi;
            const float wx = mv.x - vb.x, wy = mv.y - vb.y, wz = mv.z - vb.z;
            const float vr = fmaf(wx, dx, fmaf(wy, dy, wz * dz));
            float Pi = 0.0f;
            if (vr < 0.0f) {
                const float mu = hab * vr * __builtin_amdgcn_rcpf(fmaf(epf * hab, hab, r2));
                Pi = fmaf(-alf * 0.5f * (mt.z + tb.z), mu, bef * mu * mu) * __builtin_amdgcn_rcpf(0.5f * (mt.x + tb.x));
            }
            const float term = vb.w * ((mt.y + tb.y) + Pi) * gw;
            sx.add(-term * dx);
            sy.add(-term * dy);
            sz.add(-term * dz);
            su.add(vb.w * fmaf(0.5f, Pi, mt.y) * gw * vr);
        }
        fx = sx.value(); fy = sy.value(); fz = sz.value(); fu = su.value();
    }
    fx = lanes_sum_d(fx, gsz);
    fy = lanes_sum_d(fy, gsz);
    fz = lanes_sum_d(fz, gsz);
    fu = lanes_sum_d(fu, gsz);
    if (tv && phi == 0) {
        ax[q] = fx;
        ay[q] = fy;
        az[q] = fz;
        du[q] = fu;
    }
    }
}

void launch_forces(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double alpha, double beta,
                   double eps_av, const double*, const double*, const double*) {
    if (dm.n <= 0) return;
    if (fp32c)
        hipLaunchKernelGGL(k_forces<true>, dim3(dm.group_grid / 4 > 8 ? (dm.group_grid / 4) & ~7 : 8), dim3(256), 0, s, d.ctl, d.group, dm.group_size, dm.nbr_cap,
                           d.nbr, d.nbr_cnt, d.pos4, d.vel4, d.thr4, d.velf, d.thrf, alpha, beta, eps_av, d.ax, d.ay,
                           d.az, d.du);
    else
        hipLaunchKernelGGL(k_forces<false>, dim3(dm.group_grid / 4 > 8 ? (dm.group_grid / 4) & ~7 : 8), dim3(256), 0, s, d.ctl, d.group, dm.group_size, dm.nbr_cap,
                           d.nbr, d.nbr_cnt, d.pos4, d.vel4, d.thr4, d.velf, d.thrf, alpha, beta, eps_av, d.ax, d.ay,
                           d.az, d.du);
}
