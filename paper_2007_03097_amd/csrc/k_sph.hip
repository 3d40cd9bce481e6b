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
// One wavefront per group of group_size targets; target t is served by 64/group_size
// lanes that take every (64/group_size)-th entry of its neighbour list, then combine in a
// fixed butterfly order, so results are bitwise reproducible.  The pair sums are not a
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
__global__ void __launch_bounds__(64) k_density(const DevCtl* __restrict__ ctl, const int4* __restrict__ group,
                                                int gsz, int cap, const int* __restrict__ nbr,
                                                const int* __restrict__ nbr_cnt, double4* __restrict__ rec,
                                                RecF* __restrict__ recf, const double* __restrict__ u_eos,
                                                double gamma, double h_coeff, double* __restrict__ rho,
                                                double* __restrict__ P, double* __restrict__ cs,
                                                double* __restrict__ hnext) {
    const int lane = lane_id();
    const int t = lane & (gsz - 1), phi = lane / gsz, P_ = 64 / gsz;
    const double* recd = (const double*)rec;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
        const int4 g = group[gi];
        const bool tv = t < g.y;
        const int q = g.x + t;
        const int cnt = tv ? nbr_cnt[q] : 0;
        const int* lst = nbr + (size_t)g.x * cap + t;
        double acc, mq = 0.0, hq = 1.0;
        if (!FP32C) {
            const double4 me = tv ? rec[4 * (size_t)q] : make_double4(0, 0, 0, 1);
            mq = tv ? recd[16 * (size_t)q + 4] : 0.0;
            hq = me.w;
            double s = 0.0;
            for (int k = phi; k < cnt; k += P_) {
                const int b = lst[k * g.y];
                const double4 sb = rec[4 * (size_t)b];
                const double mb = recd[16 * (size_t)b + 4];
                const double dx = me.x - sb.x, dy = me.y - sb.y, dz = me.z - sb.z;
                const double r = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
                const double ih = 1.0 / (0.5 * (me.w + sb.w));
                s = fma(mb * m4_w(r * ih), ih * ih * ih, s);
            }
            acc = s;
        } else {
            double mx = 0, my = 0, mz = 0;
            float hf = 1.0f;
            if (tv) {
                const RecF& r = recf[q];
                mx = r.x; my = r.y; mz = r.z; hf = r.h;
                mq = (double)r.m;
            }
            Kahan s;
            for (int k = phi; k < cnt; k += P_) {
                const int b = lst[k * g.y];
                const RecF& sb = recf[b];
                const float dx = (float)(mx - sb.x), dy = (float)(my - sb.y), dz = (float)(mz - sb.z);
                const float r = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
                const float ih = __builtin_amdgcn_rcpf(0.5f * (hf + sb.h));
                s.add(sb.m * m4_wf(r * ih) * (ih * ih * ih));
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
            const double m_ = FP32C ? (double)recf[q].m : mq;
            rho[q] = r_;
            P[q] = p_;
            cs[q] = c_;
            hnext[q] = h_coeff * cbrt((FP32C ? recd[16 * (size_t)q + 4] : m_) / r_);
            rec[4 * (size_t)q + 1] = make_double4(recd[16 * (size_t)q + 4], r_, pr2, c_);
            RecF& f = recf[q];
            f.rho = (float)r_;
            f.pr2 = (float)pr2;
            f.c = (float)c_;
        }
    }
}

void launch_density(hipStream_t s, const DevPtrs& d, const Dims& dm, int fp32c, double gamma, double h_coeff,
                    const double* u_eos) {
    if (dm.n <= 0) return;
    if (fp32c)
        hipLaunchKernelGGL(k_density<true>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size,
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.rec, d.recf, u_eos, gamma, h_coeff, d.rho, d.P, d.cs,
                           d.hnext);
    else
        hipLaunchKernelGGL(k_density<false>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size,
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.rec, d.recf, u_eos, gamma, h_coeff, d.rho, d.P, d.cs,
                           d.hnext);
}

// rho, P, c given by the caller (caller order) -> key-ordered records
__global__ void k_thermo_from_caller(int n, const u32* __restrict__ id, const double* __restrict__ m,
                                     const double* __restrict__ rho, const double* __restrict__ P,
                                     const double* __restrict__ cs, double* drho, double* dP, double* dcs,
                                     double4* rec, RecF* recf) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 i = id[q];
    const double r_ = rho[i], p_ = P[i], c_ = cs[i];
    const double pr2 = p_ / (r_ * r_);
    drho[q] = r_;
    dP[q] = p_;
    dcs[q] = c_;
    rec[4 * (size_t)q + 1] = make_double4(m[q], r_, pr2, c_);
    recf[q].rho = (float)r_;
    recf[q].pr2 = (float)pr2;
    recf[q].c = (float)c_;
}

void launch_thermo_from_caller(hipStream_t s, const DevPtrs& d, const Dims& dm, const double* rho, const double* P,
                               const double* cs) {
    if (dm.n > 0)
        hipLaunchKernelGGL(k_thermo_from_caller, dim3((dm.n + 255) / 256), dim3(256), 0, s, dm.n, d.id, d.m, rho, P,
                           cs, d.rho, d.P, d.cs, d.rec, d.recf);
}

// ---------------------------------------------------------------------------------------
template <bool FP32C>
__global__ void __launch_bounds__(64) k_forces(const DevCtl* __restrict__ ctl, const int4* __restrict__ group,
                                               int gsz, int cap, const int* __restrict__ nbr,
                                               const int* __restrict__ nbr_cnt, const double4* __restrict__ rec,
                                               const RecF* __restrict__ recf, double alpha, double beta,
                                               double eps_av, double* __restrict__ ax, double* __restrict__ ay,
                                               double* __restrict__ az, double* __restrict__ du) {
    const int lane = lane_id();
    const int t = lane & (gsz - 1), phi = lane / gsz, P_ = 64 / gsz;
    int g0, g1, gstep;
    group_range(ctl->n_groups, g0, g1, gstep);
    for (int gi = g0; gi < g1; gi += gstep) {
        const int4 g = group[gi];
        const bool tv = t < g.y;
        const int q = g.x + t;
        const int cnt = tv ? nbr_cnt[q] : 0;
        const int* lst = nbr + (size_t)g.x * cap + t;
        double fx, fy, fz, fu;
        if (!FP32C) {
            const double4 me = tv ? rec[4 * (size_t)q] : make_double4(0, 0, 0, 1);
            const double4 mt = tv ? rec[4 * (size_t)q + 1] : make_double4(0, 1, 0, 0);   // m, rho, P/rho^2, c
            const double4 mv = tv ? rec[4 * (size_t)q + 2] : make_double4(0, 0, 0, 0);
            double sx = 0, sy = 0, sz = 0, su = 0;
            for (int k = phi; k < cnt; k += P_) {
                const int b = lst[k * g.y];
                const double4 sb = rec[4 * (size_t)b];
                const double4 tb = rec[4 * (size_t)b + 1];
                const double4 vb = rec[4 * (size_t)b + 2];
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
                    Pi = fma(-alpha * 0.5 * (mt.w + tb.w), mu, beta * mu * mu) / (0.5 * (mt.y + tb.y));
                }
                const double term = tb.x * ((mt.z + tb.z) + Pi) * gw;
                sx = fma(-term, dx, sx);
                sy = fma(-term, dy, sy);
                sz = fma(-term, dz, sz);
                su = fma(tb.x * fma(0.5, Pi, mt.z) * gw, vr, su);
            }
            fx = sx; fy = sy; fz = sz; fu = su;
        } else {
            double mx = 0, my = 0, mz = 0;
            float mh = 1.f, mrho = 1.f, mpr2 = 0.f, mc = 0.f, mvx = 0.f, mvy = 0.f, mvz = 0.f;
            if (tv) {
                const RecF& r = recf[q];
                mx = r.x; my = r.y; mz = r.z; mh = r.h; mrho = r.rho; mpr2 = r.pr2; mc = r.c;
                mvx = r.vx; mvy = r.vy; mvz = r.vz;
            }
            const float alf = (float)alpha, bef = (float)beta, epf = (float)eps_av;
            const float ipi = (float)M_1_PI_D;
            Neumaier sx, sy, sz, su;
            for (int k = phi; k < cnt; k += P_) {
                const int b = lst[k * g.y];
                const RecF& sb = recf[b];
                const float dx = (float)(mx - sb.x), dy = (float)(my - sb.y), dz = (float)(mz - sb.z);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float r = __builtin_amdgcn_sqrtf(r2);
                const float hab = 0.5f * (mh + sb.h);
                const float ih = __builtin_amdgcn_rcpf(hab);
                const float ih2 = ih * ih;
                const float qq = r * ih;
                const float gw = m4_gf(qq, __builtin_amdgcn_rcpf(qq)) * (ih2 * ih2 * ih) * ipi;
                const float wx = mvx - sb.vx, wy = mvy - sb.vy, wz = mvz - sb.vz;
                const float vr = fmaf(wx, dx, fmaf(wy, dy, wz * dz));
                float Pi = 0.0f;
                if (vr < 0.0f) {
                    const float mu = hab * vr * __builtin_amdgcn_rcpf(fmaf(epf * hab, hab, r2));
                    Pi = fmaf(-alf * 0.5f * (mc + sb.c), mu, bef * mu * mu) * __builtin_amdgcn_rcpf(0.5f * (mrho + sb.rho));
                }
                const float term = sb.m * ((mpr2 + sb.pr2) + Pi) * gw;
                sx.add(-term * dx);
                sy.add(-term * dy);
                sz.add(-term * dz);
                su.add(sb.m * fmaf(0.5f, Pi, mpr2) * gw * vr);
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
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.rec, d.recf, alpha, beta, eps_av, d.ax, d.ay, d.az, d.du);
    else
        hipLaunchKernelGGL(k_forces<false>, dim3(dm.group_grid), dim3(64), 0, s, d.ctl, d.group, dm.group_size,
                           dm.nbr_cap, d.nbr, d.nbr_cnt, d.rec, d.recf, alpha, beta, eps_av, d.ax, d.ay, d.az, d.du);
}
