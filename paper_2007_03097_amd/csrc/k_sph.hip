// SPH momentum and energy pair sums (Sec. 2.2.1 of arXiv:2007.03097).  The density, EOS and
// h_next (eqs. (7), (9)) are summed inside the neighbour-list kernel (k_walk.hip).
//
//   momentum (eq. (6)): dv_a/dt = -sum_b m_b ((P_a/rho_a^2 + P_b/rho_b^2) + Pi_ab) grad_a W_ab
//   energy (eq. (5)):   du_a/dt =  sum_b m_b (P_a/rho_a^2 + Pi_ab/2) v_ab . grad_a W_ab
//   viscosity:          Pi_ab = (-alpha cbar mu + beta mu^2)/rhobar if v_ab . r_ab < 0,
//                       mu = h_ab v_ab . r_ab / (r^2 + eps h_ab^2)
// with the M4 cubic spline, grad_a W_ab = r_ab g(q)/(pi h^5), g = w'(q)/q.
//
// One wavefront per group of group_size targets; target t is served by 64/group_size
// lanes that take every (64/group_size)-th entry of its neighbour list, then combine in a
// fixed butterfly order, so results are bitwise reproducible.  The pair sums are not a
// dense contraction (each target has its own irregular list), so they run on the vector
// ALUs, not on the matrix cores.
//
// FP32C: the position difference is formed in FP64 and rounded to FP32; everything else
// of the pair term is FP32, summed per lane with Neumaier compensation; lanes combine in
// FP64 and results are stored in FP64.
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

template <bool FP32C>
__global__ void __launch_bounds__(64) k_forces(const DevCtl* __restrict__ ctl, const int4* __restrict__ group,
                                               int gsz, int cap, const int* __restrict__ nbr,
                                               const int* __restrict__ nbr_cnt, const double4* __restrict__ pos4,
                                               const double4* __restrict__ vel4, const double4* __restrict__ thr4,
                                               const float4* __restrict__ velf, const float4* __restrict__ thrf,
                                               double alpha, double beta, double eps_av, double* __restrict__ ax,
                                               double* __restrict__ ay, double* __restrict__ az,
                                               double* __restrict__ du) {
    const int lane = lane_id();
    const int t = lane & (gsz - 1), phi = lane / gsz, P_ = 64 / gsz;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
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
        hipLaunchKernelGGL(k_forces<true>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size,
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.pos4, d.vel4, d.thr4, d.velf, d.thrf, alpha, beta, eps_av,
                           d.ax, d.ay, d.az, d.du);
    else
        hipLaunchKernelGGL(k_forces<false>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size,
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.pos4, d.vel4, d.thr4, d.velf, d.thrf, alpha, beta, eps_av,
                           d.ax, d.ay, d.az, d.du);
}
