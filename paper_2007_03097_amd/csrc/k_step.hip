// Leapfrog step support (kick-drift-kick with velocity and energy predictors), reordering
// of the resident state between steps, diagnostics and caller-order copies.  All FP64.
#include "common.h"

static inline dim3 g256(int n) { return dim3((n + 255) / 256); }

__global__ void k_scatter_caller(int n, const u32* __restrict__ id, const double* __restrict__ src, double* dst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[id[q]] = src[q];
}
void launch_scatter_caller(hipStream_t s, const DevPtrs& d, int n, const double* src, double* dst) {
    if (n > 0 && dst) hipLaunchKernelGGL(k_scatter_caller, g256(n), dim3(256), 0, s, n, d.id, src, dst);
}

__global__ void k_fill_zero(int n, double* dst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = 0.0;
}
void launch_fill_zero(hipStream_t s, int n, double* dst) {
    if (n > 0 && dst) hipLaunchKernelGGL(k_fill_zero, g256(n), dim3(256), 0, s, n, dst);
}

__global__ void k_gather_caller(int n, const u32* __restrict__ id, const double* __restrict__ src, double* dst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = src[id[q]];
}
void launch_gather_caller(hipStream_t s, const DevPtrs& d, int n, const double* src_caller, double* dst) {
    if (n > 0) hipLaunchKernelGGL(k_gather_caller, g256(n), dim3(256), 0, s, n, d.id, src_caller, dst);
}

// v' = v + dt/2 a; u' = u + dt/2 du; x += dt v'; predictors v^ = v' + dt/2 a, u^ = u' + dt/2 du.
// One block per chunk (chunks never cross a segment; dt is the segment's step size); the new
// positions' box is merged into the segment's box on the way, and non-finite new x, v' or u'
// raise the sticky error.  PRE: inside a run of steps, the previous step's closing half kick
// v = v + dt/2 a, u = u + dt/2 du (the same accelerations: the two kicks of the leapfrog's
// joint) and its lagged h update are applied here first, in registers, with the same roundings
// as in a separate pass.
template <bool PRE>
__global__ void __launch_bounds__(256) k_kick_drift(DevCtl* ctl, const int4* __restrict__ chunk, double* x,
                                                    double* y, double* z, double* vx, double* vy, double* vz, double* u,
                                                    const double* __restrict__ ax, const double* __restrict__ ay,
                                                    const double* __restrict__ az, const double* __restrict__ du,
                                                    double* vpx, double* vpy, double* vpz, double* up, double* h,
                                                    const double* __restrict__ hnext, int adaptive) {
    const int4 ch = chunk[blockIdx.x];
    const double dt = ctl->seg_dt[ch.z];
    const double half = 0.5 * dt;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int q = ch.x + threadIdx.x; q < ch.y; q += blockDim.x) {
        const double a0 = ax[q], a1 = ay[q], a2 = az[q], d0 = du[q];
        double v0 = vx[q], v1 = vy[q], v2 = vz[q], e0 = u[q];
        if constexpr (PRE) {
            v0 = v0 + half * a0;
            v1 = v1 + half * a1;
            v2 = v2 + half * a2;
            e0 = e0 + half * d0;
            if (adaptive) h[q] = hnext[q];
        }
        const double hx = v0 + half * a0, hy = v1 + half * a1, hz = v2 + half * a2;
        const double uh = e0 + half * d0;
        const double nx = x[q] + dt * hx, ny = y[q] + dt * hy, nz = z[q] + dt * hz;
        x[q] = nx;
        y[q] = ny;
        z[q] = nz;
        vx[q] = hx; vy[q] = hy; vz[q] = hz;
        u[q] = uh;
        vpx[q] = hx + half * a0;
        vpy[q] = hy + half * a1;
        vpz[q] = hz + half * a2;
        up[q] = uh + half * d0;
        lo[0] = fmin(lo[0], nx); lo[1] = fmin(lo[1], ny); lo[2] = fmin(lo[2], nz);
        hi[0] = fmax(hi[0], nx); hi[1] = fmax(hi[1], ny); hi[2] = fmax(hi[2], nz);
        bad |= !isfinite(nx) || !isfinite(ny) || !isfinite(nz) || !isfinite(hx) || !isfinite(hy) ||
               !isfinite(hz) || !isfinite(uh);
    }
    if (bad) set_err(ctl, ERR_NONFINITE);
    box_block_merge(ctl, ch.z, lo, hi, ch.y > ch.x);
}
void launch_kick_drift(hipStream_t s, const DevPtrs& d, const Dims& dm, bool pre_kick, int adaptive_h) {
    if (dm.n_chunks <= 0) return;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(dm.n_chunks), dim3(256), 0, s, d.ctl, d.chunk, d.x, d.y, d.z, d.vx, d.vy, d.vz,
                           d.u, d.ax, d.ay, d.az, d.du, d.vpx, d.vpy, d.vpz, d.up, d.h, d.hnext, adaptive_h);
    };
    if (pre_kick) go(k_kick_drift<true>);
    else go(k_kick_drift<false>);
}

// New key order: q <- old position val[q] (the sort carried the positions); the second
// buffer set receives the data, and the pair kernels' records pos4 = (x, h),
// vel4 = (predicted v, m) are written too.  The predicted velocities enter vel4 only: the
// next kick-drift writes them anew before anything reads them.  The step's keys are made, so
// block 0 also resets the box accumulators of every set for the next step's kick-drift (a run's
// first step resets them itself: other calls may use them in between).
__global__ void k_step_permute(int n, const u32* __restrict__ val, DevPtrs d) {
    if (blockIdx.x == 0) {
        constexpr int NB = (int)(sizeof(d.ctl->box_enc) / sizeof(u64));
        for (int i = threadIdx.x; i < NB; i += blockDim.x) d.ctl->box_enc[i] = (i % 6) < 3 ? ~0ull : 0ull;
    }
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 p = val[q];
    d.id2[q] = d.id[p];
    const double px = d.x[p], py = d.y[p], pz = d.z[p], hh = d.h[p], mm = d.m[p];
    const double wx = d.vpx[p], wy = d.vpy[p], wz = d.vpz[p];
    d.x2[q] = px; d.y2[q] = py; d.z2[q] = pz;
    d.vx2[q] = d.vx[p]; d.vy2[q] = d.vy[p]; d.vz2[q] = d.vz[p];
    d.u2[q] = d.u[p]; d.m2[q] = mm; d.h2[q] = hh;
    d.up2[q] = d.up[p];
    d.pos4[q] = make_double4(px, py, pz, hh);
    d.vel4[q] = make_double4(wx, wy, wz, mm);
}
void launch_step_permute(hipStream_t s, const DevPtrs& d, int n) {
    if (n > 0) hipLaunchKernelGGL(k_step_permute, g256(n), dim3(256), 0, s, n, d.val_a, d);
}

// v = v' + dt/2 a_new;  u = u' + dt/2 du_new;  optional lagged h update.  One block per
// chunk, dt the segment's step size.
__global__ void __launch_bounds__(256) k_kick(const DevCtl* __restrict__ ctl, const int4* __restrict__ chunk,
                                              double* vx, double* vy, double* vz, double* u,
                                              const double* __restrict__ ax, const double* __restrict__ ay,
                                              const double* __restrict__ az, const double* __restrict__ du, double* h,
                                              const double* __restrict__ hnext, int adaptive) {
    const int4 ch = chunk[blockIdx.x];
    const double half = 0.5 * ctl->seg_dt[ch.z];
    for (int q = ch.x + threadIdx.x; q < ch.y; q += blockDim.x) {
        vx[q] = vx[q] + half * ax[q];
        vy[q] = vy[q] + half * ay[q];
        vz[q] = vz[q] + half * az[q];
        u[q] = u[q] + half * du[q];
        if (adaptive) h[q] = hnext[q];
    }
}
void launch_kick(hipStream_t s, const DevPtrs& d, const Dims& dm, int adaptive_h) {
    if (dm.n_chunks > 0)
        hipLaunchKernelGGL(k_kick, dim3(dm.n_chunks), dim3(256), 0, s, d.ctl, d.chunk, d.vx, d.vy, d.vz, d.u, d.ax,
                           d.ay, d.az, d.du, d.h, d.hnext, adaptive_h);
}

__global__ void k_set_hnext(int n, double* h, const double* __restrict__ hnext) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) h[q] = hnext[q];
}
void launch_set_hnext(hipStream_t s, const DevPtrs& d, int n) {
    if (n > 0) hipLaunchKernelGGL(k_set_hnext, g256(n), dim3(256), 0, s, n, d.h, d.hnext);
}

// Diagnostics: Px, Py, Pz, Lx, Ly, Lz, Ekin, Eth, Egrav -- two fixed-order stages.
constexpr int DIAG_BLOCKS = 256;
__global__ void __launch_bounds__(256) k_diag1(int n, const double* __restrict__ x, const double* __restrict__ y,
                                                const double* __restrict__ z, const double* __restrict__ vx,
                                                const double* __restrict__ vy, const double* __restrict__ vz,
                                                const double* __restrict__ m, const double* __restrict__ u,
                                                const double* __restrict__ phi, int kin, double* part) {
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const double mm = m[q], px = x[q], py = y[q], pz = z[q], wx = vx[q], wy = vy[q], wz = vz[q];
        const double uq = kin ? u[q] - 0.5 * (wx * wx + wy * wy + wz * wz) : u[q];
        a[0] += mm * wx; a[1] += mm * wy; a[2] += mm * wz;
        a[3] += mm * (py * wz - pz * wy);
        a[4] += mm * (pz * wx - px * wz);
        a[5] += mm * (px * wy - py * wx);
        a[6] += 0.5 * mm * (wx * wx + wy * wy + wz * wz);
        a[7] += mm * uq;
        if (phi) a[8] += 0.5 * mm * phi[q];
    }
    __shared__ double red[4][9];
    const int w = threadIdx.x >> 6;
    for (int k = 0; k < 9; ++k) {
        double v = a[k];
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane_id() == 0) red[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) part[blockIdx.x * 16 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                                red[2][threadIdx.x]) + red[3][threadIdx.x];
}
__global__ void k_diag2(const double* __restrict__ part, DevCtl* ctl, int n_seg) {
    if (threadIdx.x < 9) {
        double s = 0.0;
        for (int b = 0; b < DIAG_BLOCKS; ++b) s += part[b * 16 + threadIdx.x];
        ctl->diag[threadIdx.x] = s;
    } else if (threadIdx.x == 9) {  // smallest time-step bound over the segments
        double b = INFINITY;
        for (int k = 0; k < n_seg; ++k) b = fmin(b, dec_double(ctl->dtb_enc[k]));
        ctl->diag[9] = b;
    }
}
// Diagnostics of the resident state plus (diag[9]) the time-step bound of k_dt_bound.
void launch_diag(hipStream_t s, const DevPtrs& d, const Dims& dm, int with_phi, int kin, double eps_grav) {
    launch_dt_bound(s, d, dm, eps_grav);
    hipLaunchKernelGGL(k_diag1, dim3(DIAG_BLOCKS), dim3(256), 0, s, dm.n, d.x, d.y, d.z, d.vx, d.vy, d.vz, d.m, d.u,
                       with_phi ? d.phi : nullptr, kin, d.diag_part);
    hipLaunchKernelGGL(k_diag2, dim3(1), dim3(64), 0, s, d.diag_part, d.ctl, dm.n_seg);
}

// Resident key-ordered state -> caller order (kin: the resident u is e = u + v^2/2).
__global__ void k_write_back(int n, DevPtrs d, double* x, double* y, double* z, double* vx, double* vy, double* vz,
                             double* h, double* u, double* ax, double* ay, double* az, double* du, int kin) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 i = d.id[q];
    const double wx = d.vx[q], wy = d.vy[q], wz = d.vz[q];
    x[i] = d.x[q]; y[i] = d.y[q]; z[i] = d.z[q];
    vx[i] = wx; vy[i] = wy; vz[i] = wz;
    h[i] = d.h[q];
    u[i] = kin ? d.u[q] - 0.5 * (wx * wx + wy * wy + wz * wz) : d.u[q];
    if (ax) { ax[i] = d.ax[q]; ay[i] = d.ay[q]; az[i] = d.az[q]; du[i] = d.du[q]; }
}
void launch_write_back(hipStream_t s, const DevPtrs& d, int n, double* x, double* y, double* z, double* vx, double* vy,
                       double* vz, double* h, double* u, double* ax, double* ay, double* az, double* du, int kin) {
    if (n > 0)
        hipLaunchKernelGGL(k_write_back, g256(n), dim3(256), 0, s, n, d, x, y, z, vx, vy, vz, h, u, ax, ay, az, du,
                           kin);
}

// Thermokinetic form: the resident thermal u becomes the total energy e = u + v^2/2.
__global__ void k_add_kinetic(int n, const double* __restrict__ vx, const double* __restrict__ vy,
                              const double* __restrict__ vz, double* u) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double wx = vx[q], wy = vy[q], wz = vz[q];
    u[q] = u[q] + 0.5 * (wx * wx + wy * wy + wz * wz);
}
void launch_add_kinetic(hipStream_t s, const DevPtrs& d, int n) {
    if (n > 0) hipLaunchKernelGGL(k_add_kinetic, g256(n), dim3(256), 0, s, n, d.vx, d.vy, d.vz, d.u);
}

// Caller-supplied accelerations of the input state -> key order.
__global__ void k_load_accel(int n, const u32* __restrict__ id, const double* __restrict__ ax,
                             const double* __restrict__ ay, const double* __restrict__ az,
                             const double* __restrict__ du, double* dax, double* day, double* daz, double* ddu) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 i = id[q];
    dax[q] = ax[i]; day[q] = ay[i]; daz[q] = az[i]; ddu[q] = du[i];
}
void launch_load_accel(hipStream_t s, const DevPtrs& d, int n, const double* ax, const double* ay, const double* az,
                       const double* du) {
    if (n > 0) hipLaunchKernelGGL(k_load_accel, g256(n), dim3(256), 0, s, n, d.id, ax, ay, az, du, d.ax, d.ay, d.az, d.du);
}

// Time-step bound of the resident state, per segment: min over its particles of
// min(h/c, sqrt(eps/|a|)) (the second term only when eps > 0, i.e. with self-gravity and
// softening; |a| = 0 gives no bound).  h is the current smoothing length, c the sound speed
// of the last density pass, a the last accelerations.  A minimum is exact in any order, so
// the chunks merge into the segment's value with atomics on the ordered-integer encoding.
__global__ void k_dt_bound_init(DevCtl* ctl, int n_seg) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_seg) ctl->dtb_enc[s] = enc_double(INFINITY);
}
__global__ void __launch_bounds__(256) k_dt_bound(DevCtl* ctl, const int4* __restrict__ chunk,
                                                  const double* __restrict__ h, const double* __restrict__ cs,
                                                  const double* __restrict__ ax, const double* __restrict__ ay,
                                                  const double* __restrict__ az, double eps) {
    const int4 ch = chunk[blockIdx.x];
    double b = INFINITY;
    for (int q = ch.x + threadIdx.x; q < ch.y; q += blockDim.x) {
        double v = h[q] / cs[q];
        if (eps > 0.0) {
            const double a0 = ax[q], a1 = ay[q], a2 = az[q];
            const double a = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
            if (a > 0.0) v = fmin(v, sqrt(eps / a));
        }
        b = fmin(b, v);
    }
    b = wave_min(b);
    __shared__ double red[4];
    if (lane_id() == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        if (ch.y > ch.x) atomicMin(&ctl->dtb_enc[ch.z], enc_double(m));
    }
}
void launch_dt_bound(hipStream_t s, const DevPtrs& d, const Dims& dm, double eps_grav) {
    hipLaunchKernelGGL(k_dt_bound_init, dim3((dm.n_seg + 255) / 256), dim3(256), 0, s, d.ctl, dm.n_seg);
    if (dm.n_chunks > 0)
        hipLaunchKernelGGL(k_dt_bound, dim3(dm.n_chunks), dim3(256), 0, s, d.ctl, d.chunk, d.h, d.cs, d.ax, d.ay, d.az,
                           eps_grav);
}

// Keys (caller order) and key order of the resident state: the sorted keys of the last key
// sort, and the caller index of each sorted position.
__global__ void k_resident_export(int n, const u32* __restrict__ id, const u64* __restrict__ skey, u64* keys,
                                  int64_t* order) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const u32 i = id[q];
    if (keys) keys[i] = skey[q];
    if (order) order[q] = (int64_t)i;
}
void launch_resident_export(hipStream_t s, const DevPtrs& d, int n, u64* keys_caller, int64_t* order) {
    if (n > 0) hipLaunchKernelGGL(k_resident_export, g256(n), dim3(256), 0, s, n, d.id, d.key_a, keys_caller, order);
}
