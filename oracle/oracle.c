/*
 * oracle.c -- plain, slow, obviously correct CPU reference (FP64) for the SPH + octree
 * hot path of FleCSPH (arXiv:2007.03097).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this code.  It shares no source, header, table or helper with
 * the GPU library; the two meet only through seeded inputs.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction, so every
 * product and sum below is one IEEE operation in the order written).
 *
 * Conventions (readings of the paper where it is silent; each is listed with its reason
 * in the design notes):
 *   - keys: 21 bits per axis, x in the lowest bit of every 3-bit digit, a leading 1
 *     ("sentinel") above the digits (Sec. 2.1 "Tree topology", Fig. 1).  Sets split into
 *     segments use 18 bits per axis and put the segment number in the three digits just
 *     below the sentinel.
 *   - smoothing kernel: M4 cubic spline, support 2h, sigma = 1/pi in 3D; every pair uses
 *     h_ab = (h_a + h_b)/2 (text after eq. (6)), also in the density sum (eq. (7)), and the
 *     density sum includes the particle itself.
 *   - neighbours of a: every b with |r_a - r_b| < h_a + h_b (= 2 h_ab), decided by
 *     fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)) < fl(t*t), t = fl(h_a + h_b).
 *   - artificial viscosity: Monaghan form with mu = h_ab v_ab.r_ab / (r^2 + eps h_ab^2),
 *     Pi = (-alpha cbar mu + beta mu^2) / rhobar for approaching pairs, else 0.
 *   - gravity: Plummer-softened Newtonian sums (eq. (10) with softening); the tree
 *     reference uses monopole + quadrupole about each accepted cell's centre of mass.
 *
 * Parity pins for every function are in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------ */
/* Keys (Sec. 2.1, "Tree topology"; Fig. 1): quantise each coordinate to B bits inside the
 * cubic root cell of side L = max extent, interleave the bits (x lowest), prefix the
 * sentinel.  box: per segment lo_x, lo_y, lo_z, hi_x, hi_y, hi_z.                        */

static uint64_t orc_interleave(uint32_t kx, uint32_t ky, uint32_t kz, int bits)
{
    uint64_t key = 0;
    for (int l = 0; l < bits; ++l) {
        key |= (uint64_t)((kx >> l) & 1u) << (3 * l);
        key |= (uint64_t)((ky >> l) & 1u) << (3 * l + 1);
        key |= (uint64_t)((kz >> l) & 1u) << (3 * l + 2);
    }
    return key;
}

static uint32_t orc_quantise(double x, double lo, double S, int bits)
{
    double t = (x - lo) * S;               /* one subtraction, one multiplication */
    uint32_t top = (1u << bits) - 1u;
    if (!(t > 0.0)) return 0u;             /* also catches t == 0 */
    if (t >= (double)top) return top;
    return (uint32_t)t;                    /* truncation */
}

/* Exact bounding box of particles [b, e). */
void orc_bbox(int64_t b, int64_t e, const double* x, const double* y, const double* z, double* box6)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const double* c[3] = {x, y, z};
    for (int64_t i = b; i < e; ++i)
        for (int d = 0; d < 3; ++d) {
            if (c[d][i] < lo[d]) lo[d] = c[d][i];
            if (c[d][i] > hi[d]) hi[d] = c[d][i];
        }
    for (int d = 0; d < 3; ++d) { box6[d] = lo[d]; box6[3 + d] = hi[d]; }
}

/* Scale S = 2^B / L with L the largest extent; 0 when L is 0 or the quotient overflows. */
double orc_scale(const double* box6, int bits)
{
    double L = 0.0;
    for (int d = 0; d < 3; ++d) {
        double ext = box6[3 + d] - box6[d];
        if (ext > L) L = ext;
    }
    if (!(L > 0.0)) return 0.0;
    double S = ldexp(1.0, bits) / L;
    return isfinite(S) ? S : 0.0;
}

/* Keys for n particles in caller order.  nseg <= 1 and seg_off == NULL: one set (B = 21).
 * Otherwise segments [seg_off[s], seg_off[s+1]) with B = 18 and the segment number in
 * bits 54..62.  box (6 per segment) may be NULL: then each segment's exact bbox is used. */
void orc_keys(int64_t n, const double* x, const double* y, const double* z, int32_t nseg,
              const int64_t* seg_off, const double* box, uint64_t* keys)
{
    int batched = (nseg > 1);
    int bits = batched ? 18 : 21;
    int32_t ns = batched ? nseg : 1;
    for (int32_t s = 0; s < ns; ++s) {
        int64_t b = batched ? seg_off[s] : 0, e = batched ? seg_off[s + 1] : n;
        double bb[6];
        if (box) memcpy(bb, box + 6 * s, sizeof bb);
        else orc_bbox(b, e, x, y, z, bb);
        double S = orc_scale(bb, bits);
        uint64_t prefix = (1ull << 63) | (batched ? ((uint64_t)s << 54) : 0ull);
        for (int64_t i = b; i < e; ++i) {
            uint32_t kx = orc_quantise(x[i], bb[0], S, bits);
            uint32_t ky = orc_quantise(y[i], bb[1], S, bits);
            uint32_t kz = orc_quantise(z[i], bb[2], S, bits);
            keys[i] = prefix | orc_interleave(kx, ky, kz, bits);
        }
    }
}

/* 3D Hilbert index of grid cell (kx, ky, kz) on a 2^bits grid, by Skilling's transposition
 * (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 381 (2004)): the
 * coordinates are transformed into the "transposed" index in place, whose bits read out
 * level by level (x, then y, then z within a level) give the index.  One 3-bit digit per
 * level, so every octree cell is one contiguous run of indices.                          */
uint64_t orc_hilbert(uint32_t kx, uint32_t ky, uint32_t kz, int bits)
{
    uint32_t X[3] = {kx, ky, kz};
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {      /* inverse undo */
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;                        /* invert the low bits of x */
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;   /* exchange low bits of x and axis i */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1]; /* Gray encode */
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
    return h;
}

/* orc_keys with the Hilbert index in place of the bit interleave (same quantisation,
 * sentinel and segment prefix).                                                          */
void orc_keys_hilbert(int64_t n, const double* x, const double* y, const double* z, int32_t nseg,
                      const int64_t* seg_off, const double* box, uint64_t* keys)
{
    int batched = (nseg > 1);
    int bits = batched ? 18 : 21;
    int32_t ns = batched ? nseg : 1;
    for (int32_t s = 0; s < ns; ++s) {
        int64_t b = batched ? seg_off[s] : 0, e = batched ? seg_off[s + 1] : n;
        double bb[6];
        if (box) memcpy(bb, box + 6 * s, sizeof bb);
        else orc_bbox(b, e, x, y, z, bb);
        double S = orc_scale(bb, bits);
        uint64_t prefix = (1ull << 63) | (batched ? ((uint64_t)s << 54) : 0ull);
        for (int64_t i = b; i < e; ++i) {
            uint32_t kx = orc_quantise(x[i], bb[0], S, bits);
            uint32_t ky = orc_quantise(y[i], bb[1], S, bits);
            uint32_t kz = orc_quantise(z[i], bb[2], S, bits);
            keys[i] = prefix | orc_hilbert(kx, ky, kz, bits);
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Order: sort by (key, caller index); the caller index is the paper's unique particle ID
 * that resolves key collisions (Sec. 2.1).                                               */

static const uint64_t* orc_sort_keys;
static int orc_cmp(const void* a, const void* b)
{
    int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
    uint64_t ki = orc_sort_keys[i], kj = orc_sort_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return (i > j) - (i < j);
}

void orc_order(int64_t n, const uint64_t* keys, int64_t* order)
{
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    orc_sort_keys = keys;
    qsort(order, (size_t)n, sizeof(int64_t), orc_cmp);
}

/* ------------------------------------------------------------------------------------ */
/* Octree (Sec. 2.1: particles are inserted and cells refined into 2^D children until every
 * particle is isolated; here "isolated" generalises to at most leaf_cap particles).  The
 * tree is built top-down over the sorted keys.  Output in pre-order: node key (sentinel
 * bit 3*level followed by the level's digits), level, leaf flag, first sorted position,
 * particle count.  Levels below min_level are always refined (used for segmented sets so
 * that every segment owns its own subtree).  Returns the node count, or -1 when cap is
 * too small.                                                                             */

typedef struct {
    const uint64_t* k;
    int leaf_cap, min_level;
    int64_t cap, count;
    uint64_t* nkey; int32_t* nlevel; int32_t* nleaf; int64_t* nstart; int64_t* ncount;
} orc_tree_ctx;

static uint64_t orc_digits(uint64_t key, int level)
{
    return level == 0 ? 0ull : ((key & ~(1ull << 63)) >> (3 * (21 - level)));
}

static int orc_tree_rec(orc_tree_ctx* t, int level, int64_t s, int64_t e)
{
    if (t->count >= t->cap) return -1;
    int64_t me = t->count++;
    t->nkey[me] = (1ull << (3 * level)) | orc_digits(t->k[s], level);
    t->nlevel[me] = level;
    t->nstart[me] = s;
    t->ncount[me] = e - s;
    int leaf = (level >= t->min_level && e - s <= t->leaf_cap) || level == 21;
    t->nleaf[me] = leaf;
    if (leaf) return 0;
    int64_t c = s;
    while (c < e) {  /* children: runs of equal digit at level+1 */
        uint64_t d = orc_digits(t->k[c], level + 1);
        int64_t ce = c;
        while (ce < e && orc_digits(t->k[ce], level + 1) == d) ++ce;
        if (orc_tree_rec(t, level + 1, c, ce) < 0) return -1;
        c = ce;
    }
    return 0;
}

int64_t orc_octree(int64_t n, const uint64_t* sorted_keys, int leaf_cap, int min_level, int64_t cap,
                   uint64_t* nkey, int32_t* nlevel, int32_t* nleaf, int64_t* nstart, int64_t* ncount)
{
    if (n == 0) return 0;
    orc_tree_ctx t = {sorted_keys, leaf_cap, min_level, cap, 0, nkey, nlevel, nleaf, nstart, ncount};
    if (orc_tree_rec(&t, 0, 0, n) < 0) return -1;
    return t.count;
}

/* ------------------------------------------------------------------------------------ */
/* Neighbours by brute force over all pairs.  seg (int32 per particle, may be NULL) keeps
 * pairs inside one segment.  Lists are sorted by ascending caller index and include the
 * particle itself.  targets (ntgt entries, may be NULL = all particles in order).        */

static int orc_is_nbr(int64_t a, int64_t b, const double* x, const double* y, const double* z,
                      const double* h)
{
    double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    double t = h[a] + h[b];
    return r2 < t * t;
}

void orc_nbr_count(int64_t n, const double* x, const double* y, const double* z, const double* h,
                   const int32_t* seg, int64_t ntgt, const int64_t* tgt, int64_t* counts)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t a = tgt ? tgt[t] : t, c = 0;
        for (int64_t b = 0; b < n; ++b) {
            if (seg && seg[a] != seg[b]) continue;
            c += orc_is_nbr(a, b, x, y, z, h);
        }
        counts[t] = c;
    }
}

void orc_nbr_fill(int64_t n, const double* x, const double* y, const double* z, const double* h,
                  const int32_t* seg, int64_t ntgt, const int64_t* tgt, const int64_t* offsets, int64_t* idx)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t a = tgt ? tgt[t] : t, w = offsets[t];
        for (int64_t b = 0; b < n; ++b) {
            if (seg && seg[a] != seg[b]) continue;
            if (orc_is_nbr(a, b, x, y, z, h)) idx[w++] = b;
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* M4 cubic spline in 3D (the kernel family named for FleCSPH's "selection of kernels",
 * Sec. 2.2.1): W(r, h) = w(q) / (pi h^3), q = r/h,
 *   w = 1 - 1.5 q^2 + 0.75 q^3 (q < 1),  0.25 (2 - q)^3 (1 <= q < 2),  0 (q >= 2).
 * grad_a W_ab = r_ab * g(q) / (pi h^5) with g = w'(q)/q.                                 */

double orc_w(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) { double t = 2.0 - q; return 0.25 * t * t * t; }
    return 0.0;
}

double orc_dw_over_q(double q)
{
    if (q < 1.0) return -3.0 + 2.25 * q;
    if (q < 2.0) { double t = 2.0 - q; return -0.75 * t * t / q; }
    return 0.0;
}

/* Density (eq. (7)) and ideal-gas EOS over a CSR neighbour list, for ntgt targets.
 *   rho_a = sum_b m_b W(r_ab, h_ab);  P_a = (gamma - 1) rho_a u_a;  c_a = sqrt(gamma P_a / rho_a)
 *   h_next_a = h_coeff (m_a / rho_a)^(1/3)   (eq. (9) with C eta = h_coeff, D = 3)
 * out arrays are indexed by target number t.                                             */
void orc_density(const double* x, const double* y, const double* z, const double* h, const double* m,
                 const double* u, double gamma, double h_coeff, int64_t ntgt, const int64_t* tgt,
                 const int64_t* offsets, const int64_t* idx, double* rho, double* P, double* c,
                 double* h_next)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t a = tgt ? tgt[t] : t;
        double s = 0.0;
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            int64_t b = idx[k];
            double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double hab = 0.5 * (h[a] + h[b]);
            double W = orc_w(r / hab) / (ORC_PI * hab * hab * hab);
            s += m[b] * W;
        }
        rho[t] = s;
        P[t] = (gamma - 1.0) * s * u[a];
        c[t] = sqrt(gamma * P[t] / s);
        if (h_next) h_next[t] = h_coeff * cbrt(m[a] / s);
    }
}

/* Momentum (eq. (6), g = 0) and internal energy (eq. (5)) with Monaghan viscosity over a
 * CSR neighbour list (self entries skipped).  rho, P, c are indexed by particle.  Also
 * returns the absolute-sum scales used for the relative tolerance, each the sum of the
 * magnitudes of the elementary products the sum expands into (the dot product v . grad W
 * counted as its three products, whose rounding does not shrink when v is orthogonal to
 * grad W):
 *   Sa_a = sum_b m_b |(P_a/rho_a^2 + P_b/rho_b^2) + Pi_ab| |grad_a W_ab|
 *   Su_a = sum_b m_b |P_a/rho_a^2 + Pi_ab/2| sum_d |v_ab,d (grad_a W_ab)_d|                */
void orc_forces(const double* x, const double* y, const double* z, const double* vx, const double* vy,
                const double* vz, const double* h, const double* m, const double* rho, const double* P,
                const double* c, double alpha, double beta, double eps_av, int64_t ntgt, const int64_t* tgt,
                const int64_t* offsets, const int64_t* idx, double* ax, double* ay, double* az, double* dudt,
                double* Sa, double* Su)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t a = tgt ? tgt[t] : t;
        double pa = P[a] / (rho[a] * rho[a]);
        double fx = 0, fy = 0, fz = 0, du = 0, sa = 0, su = 0;
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            int64_t b = idx[k];
            if (b == a) continue;
            double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
            double r2 = dx * dx + dy * dy + dz * dz;
            double r = sqrt(r2);
            double hab = 0.5 * (h[a] + h[b]);
            double q = r / hab;
            double gw = orc_dw_over_q(q) / (ORC_PI * hab * hab * hab * hab * hab);
            double gx = dx * gw, gy = dy * gw, gz = dz * gw;  /* grad_a W_ab */
            double wx = vx[a] - vx[b], wy = vy[a] - vy[b], wz = vz[a] - vz[b];
            double vr = wx * dx + wy * dy + wz * dz;
            double Pi = 0.0;
            if (vr < 0.0) {
                double mu = hab * vr / (r2 + eps_av * hab * hab);
                double cbar = 0.5 * (c[a] + c[b]), rbar = 0.5 * (rho[a] + rho[b]);
                Pi = (-alpha * cbar * mu + beta * mu * mu) / rbar;
            }
            double pb = P[b] / (rho[b] * rho[b]);
            double term = (pa + pb) + Pi;
            fx -= m[b] * term * gx;
            fy -= m[b] * term * gy;
            fz -= m[b] * term * gz;
            double vg = wx * gx + wy * gy + wz * gz;
            du += m[b] * (pa + 0.5 * Pi) * vg;
            sa += m[b] * fabs(term) * sqrt(gx * gx + gy * gy + gz * gz);
            su += m[b] * fabs(pa + 0.5 * Pi) * (fabs(wx * gx) + fabs(wy * gy) + fabs(wz * gz));
        }
        ax[t] = fx; ay[t] = fy; az[t] = fz; dudt[t] = du;
        if (Sa) Sa[t] = sa;
        if (Su) Su[t] = su;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Thermokinetic energy equation (Sec. 2.2.1, eq. (8)): the total specific energy
 * e_a = u_a + v_a^2 / 2 evolves as
 *   de_a/dt = -sum_{b != a} m_b (P_a v_b / rho_a^2 + P_b v_a / rho_b^2
 *                                + (v_a + v_b)/2 Pi_ab) . grad_a W_ab,
 * with W, h_ab and Pi_ab exactly as in orc_forces.  Se: the absolute-sum scale (for
 * relative error bounds), each dot product counted as its three products.              */
void orc_dedt(const double* x, const double* y, const double* z, const double* vx, const double* vy,
              const double* vz, const double* h, const double* m, const double* rho, const double* P,
              const double* c, double alpha, double beta, double eps_av, int64_t ntgt, const int64_t* tgt,
              const int64_t* offsets, const int64_t* idx, double* dedt, double* Se)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t a = tgt ? tgt[t] : t;
        double pa = P[a] / (rho[a] * rho[a]);
        double de = 0, se = 0;
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            int64_t b = idx[k];
            if (b == a) continue;
            double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
            double r2 = dx * dx + dy * dy + dz * dz;
            double r = sqrt(r2);
            double hab = 0.5 * (h[a] + h[b]);
            double q = r / hab;
            double gw = orc_dw_over_q(q) / (ORC_PI * hab * hab * hab * hab * hab);
            double gx = dx * gw, gy = dy * gw, gz = dz * gw;  /* grad_a W_ab */
            double wx = vx[a] - vx[b], wy = vy[a] - vy[b], wz = vz[a] - vz[b];
            double vr = wx * dx + wy * dy + wz * dz;
            double Pi = 0.0;
            if (vr < 0.0) {
                double mu = hab * vr / (r2 + eps_av * hab * hab);
                double cbar = 0.5 * (c[a] + c[b]), rbar = 0.5 * (rho[a] + rho[b]);
                Pi = (-alpha * cbar * mu + beta * mu * mu) / rbar;
            }
            double pb = P[b] / (rho[b] * rho[b]);
            double vag = vx[a] * gx + vy[a] * gy + vz[a] * gz;   /* v_a . grad_a W_ab */
            double vbg = vx[b] * gx + vy[b] * gy + vz[b] * gz;   /* v_b . grad_a W_ab */
            double t1 = pa * vbg, t2 = pb * vag, t3 = 0.5 * Pi * (vag + vbg);
            de -= m[b] * (t1 + t2 + t3);
            double avag = fabs(vx[a] * gx) + fabs(vy[a] * gy) + fabs(vz[a] * gz);
            double avbg = fabs(vx[b] * gx) + fabs(vy[b] * gy) + fabs(vz[b] * gz);
            se += m[b] * (fabs(pa) * avbg + fabs(pb) * avag + fabs(0.5 * Pi) * (avag + avbg));
        }
        dedt[t] = de;
        if (Se) Se[t] = se;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Direct-sum self-gravity (eq. (10) with theta_MAC = 0: every cell opened down to single
 * particles), Plummer softened:
 *   g_a = -G sum_{b != a} m_b r_ab / (r_ab^2 + eps^2)^{3/2},
 *   phi_a = -G sum_{b != a} m_b / sqrt(r_ab^2 + eps^2).                                   */
void orc_gravity_direct(int64_t n, const double* x, const double* y, const double* z, const double* m,
                        double G, double eps, int64_t ntgt, const int64_t* tgt, double* gx, double* gy,
                        double* gz, double* phi, double* sg)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t a = tgt ? tgt[t] : t;
        double sx = 0, sy = 0, sz = 0, sp = 0, sa = 0;
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
            double s2 = dx * dx + dy * dy + dz * dz + eps * eps;
            double inv = 1.0 / sqrt(s2);
            double inv3 = inv * inv * inv;
            sx -= m[b] * dx * inv3;
            sy -= m[b] * dy * inv3;
            sz -= m[b] * dz * inv3;
            sp -= m[b] * inv;
            if (sg) sa += m[b] * sqrt(dx * dx + dy * dy + dz * dz) * inv3;
        }
        gx[t] = G * sx; gy[t] = G * sy; gz[t] = G * sz;
        if (phi) phi[t] = G * sp;
        if (sg) sg[t] = fabs(G) * sa;   /* absolute-sum scale: sum of the terms' magnitudes */
    }
}

/* Monopole + quadrupole moments of particles idx[0..k) (or [b, e) when idx == NULL):
 * mass M, centre of mass R, second moments I = sum m y y^T with y = r - R (xx,yy,zz,xy,xz,yz). */
void orc_moments(int64_t b, int64_t e, const int64_t* idx, const double* x, const double* y,
                 const double* z, const double* m, double* out10)
{
    double M = 0, sx = 0, sy = 0, sz = 0;
    for (int64_t k = b; k < e; ++k) {
        int64_t j = idx ? idx[k] : k;
        M += m[j]; sx += m[j] * x[j]; sy += m[j] * y[j]; sz += m[j] * z[j];
    }
    double R[3] = {sx / M, sy / M, sz / M};
    double I[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = b; k < e; ++k) {
        int64_t j = idx ? idx[k] : k;
        double d[3] = {x[j] - R[0], y[j] - R[1], z[j] - R[2]};
        I[0] += m[j] * d[0] * d[0]; I[1] += m[j] * d[1] * d[1]; I[2] += m[j] * d[2] * d[2];
        I[3] += m[j] * d[0] * d[1]; I[4] += m[j] * d[0] * d[2]; I[5] += m[j] * d[1] * d[2];
    }
    out10[0] = M; out10[1] = R[0]; out10[2] = R[1]; out10[3] = R[2];
    for (int q = 0; q < 6; ++q) out10[4 + q] = I[q];
}

/* Field at point p of a cell with moments mom10, from the second-order Taylor expansion of
 * the softened potential -G m / sqrt(|p - r_j|^2 + eps^2) about the centre of mass (the
 * dipole term vanishes there).  With R = p - R_B and s^2 = |R|^2 + eps^2:
 *   phi = -G [M/s + (3/2) R.I.R / s^5 - (1/2) tr(I) / s^3]
 *   g   =  G [-M R/s^3 + 3 I.R/s^5 - (15/2)(R.I.R) R/s^7 + (3/2) tr(I) R/s^5]              */
void orc_quad_field(const double* mom10, double px, double py, double pz, double G, double eps,
                    double* g3, double* phi)
{
    double M = mom10[0];
    double R[3] = {px - mom10[1], py - mom10[2], pz - mom10[3]};
    const double* I = mom10 + 4;
    double IR[3] = {I[0] * R[0] + I[3] * R[1] + I[4] * R[2],
                    I[3] * R[0] + I[1] * R[1] + I[5] * R[2],
                    I[4] * R[0] + I[5] * R[1] + I[2] * R[2]};
    double RIR = R[0] * IR[0] + R[1] * IR[1] + R[2] * IR[2];
    double trI = I[0] + I[1] + I[2];
    double s2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2] + eps * eps;
    double s = sqrt(s2);
    double i1 = 1.0 / s, i3 = i1 / s2, i5 = i3 / s2, i7 = i5 / s2;
    for (int d = 0; d < 3; ++d)
        g3[d] = G * (-M * R[d] * i3 + 3.0 * IR[d] * i5 - 7.5 * RIR * R[d] * i7 + 1.5 * trI * R[d] * i5);
    *phi = -G * (M * i1 + 1.5 * RIR * i5 - 0.5 * trI * i3);
}

/* Tree gravity reference: the same octree as orc_octree (pre-order node list over particles
 * in sorted order), walked once per target group [gstart[g], gstart[g] + gcount[g]).
 * A cell B is accepted for the whole group when its radius b_B about its centre of mass is
 * below theta * d, d being the distance from that centre of mass to the group's bounding
 * box, and B's particle box does not touch the group's box (the paper's MAC = 1 limit: nodes
 * that do not intersect, Sec. 3.4).  b_B is the distance from the centre of mass to the
 * farthest corner of B's particle box (an upper bound of its largest particle distance; the
 * paper's opening test compares node radii with the distance, Sec. 2.2.2).  Accepted cells contribute through orc_quad_field; unaccepted
 * leaves through softened particle sums with the target itself excluded; unaccepted
 * internal cells are opened.  theta = 0 opens everything (exact direct sum, Sec. 2.2.2).
 * L (the root cell side) is not used by this opening test; it stays in the interface.
 * counts (nullable): [0] cell terms evaluated (accepted cells times their group's targets),
 * [1] particle-particle terms (each target's own pair excluded).                          */
void orc_tree_gravity(int64_t n, int64_t n_nodes, const int32_t* nlevel, const int32_t* nleaf,
                      const int64_t* nstart, const int64_t* ncount, const double* x, const double* y,
                      const double* z, const double* m, double L, double theta, double G, double eps,
                      int64_t ngroups, const int64_t* gstart, const int64_t* gcount, double* gx, double* gy,
                      double* gz, double* phi, int64_t* counts)
{
    int64_t n_cells = 0, n_pairs = 0;
    int64_t* child = (int64_t*)malloc(sizeof(int64_t) * 8 * (size_t)n_nodes);
    int32_t* nch = (int32_t*)calloc((size_t)n_nodes, sizeof(int32_t));
    double* mom = (double*)malloc(sizeof(double) * 10 * (size_t)n_nodes);
    double* nbox = (double*)malloc(sizeof(double) * 6 * (size_t)n_nodes);
    int64_t last_at_level[23];
    for (int64_t j = 0; j < n_nodes; ++j) {   /* parent = latest node one level up */
        last_at_level[nlevel[j]] = j;
        if (nlevel[j] > 0) {
            int64_t p = last_at_level[nlevel[j] - 1];
            child[8 * p + nch[p]++] = j;
        }
        orc_moments(nstart[j], nstart[j] + ncount[j], NULL, x, y, z, m, mom + 10 * j);
        orc_bbox(nstart[j], nstart[j] + ncount[j], x, y, z, nbox + 6 * j);
    }
    for (int64_t a = 0; a < n; ++a) { gx[a] = gy[a] = gz[a] = phi[a] = 0.0; }
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_cells, n_pairs)
    for (int64_t g = 0; g < ngroups; ++g) {
        int64_t g0 = gstart[g], g1 = g0 + gcount[g];
        double gb[6];
        orc_bbox(g0, g1, x, y, z, gb);
        int64_t st[256];   /* depth-first: at most 8 entries per level, 22 levels */
        int sp = 0;
        if (n_nodes > 0) st[sp++] = 0;
        while (sp > 0) {
            int64_t node = st[--sp];
            const double* nb = nbox + 6 * node;
            const double* mo = mom + 10 * node;
            double b2 = 0.0;   /* b_B^2 */
            for (int d = 0; d < 3; ++d) {
                double u = fmax(mo[1 + d] - nb[d], nb[3 + d] - mo[1 + d]);
                b2 += u * u;
            }
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                double q = mo[1 + d];
                double gap = q < gb[d] ? gb[d] - q : (q > gb[3 + d] ? q - gb[3 + d] : 0.0);
                d2 += gap * gap;
            }
            int apart = 0;
            for (int d = 0; d < 3; ++d)
                if (nb[d] > gb[3 + d] || nb[3 + d] < gb[d]) apart = 1;
            if (apart && b2 < theta * theta * d2) {
                for (int64_t a = g0; a < g1; ++a) {
                    double g3[3], p;
                    orc_quad_field(mo, x[a], y[a], z[a], G, eps, g3, &p);
                    gx[a] += g3[0]; gy[a] += g3[1]; gz[a] += g3[2]; phi[a] += p;
                    ++n_cells;
                }
            } else if (nleaf[node]) {
                int64_t b0 = nstart[node], b1 = b0 + ncount[node];
                for (int64_t a = g0; a < g1; ++a)
                    for (int64_t b = b0; b < b1; ++b) {
                        if (b == a) continue;
                        ++n_pairs;
                        double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
                        double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
                        double inv3 = inv * inv * inv;
                        gx[a] -= G * m[b] * dx * inv3;
                        gy[a] -= G * m[b] * dy * inv3;
                        gz[a] -= G * m[b] * dz * inv3;
                        phi[a] -= G * m[b] * inv;
                    }
            } else {
                for (int32_t k = nch[node] - 1; k >= 0; --k) st[sp++] = child[8 * node + k];
            }
        }
    }
    free(child); free(nch); free(mom); free(nbox);
    if (counts) { counts[0] = n_cells; counts[1] = n_pairs; }
}

/* ------------------------------------------------------------------------------------ */
/* Symmetric node-node gravity (the paper's own scheme, Sec. 2.2.2 and eq. (10), after
 * Dehnen 2000): a mutual recursion over pairs of nodes of the octree above.
 *
 *   interact(A, A): a leaf sums all its particle pairs directly; an internal node
 *                   interacts every child with itself and every unordered pair of children.
 *   interact(A, B): if the MAC accepts (A, B), one node-node term; else, if both are
 *                   leaves, every particle pair directly; else the larger node (lower level;
 *                   on equal levels the one whose particles come first in key order) is
 *                   split -- unless it is a leaf, then the other one -- and each of its
 *                   children interacts with the other node.
 *
 * MAC: every cell is enclosed by the sphere of radius (sqrt 3 / 2) side about its centre;
 * (A, B) is accepted when r_A + r_B < theta |c_A - c_B|.  The cells are the octree cells of
 * the quantised keys (cell of node j: the quantised coordinates of its first particle,
 * shifted to its level), so in units of half the finest cell every quantity is an integer:
 *   T = 2 (s_A + s_B),  D = 2 (c_A - c_B),  accept  <=>  3 T^2 < 4 theta^2 |D|^2.
 * theta = 0 never accepts: the result is the direct sum.
 *
 * Node-node term (first order in the Taylor expansion of the potential about each
 * centre of mass, with monopole sources, so the field is constant across a node; eq. (10)
 * with R_AB = R_A - R_B, Plummer softened, s^2 = |R_AB|^2 + eps^2):
 *   node A:  g += -G M_B R_AB / s^3,  phi(R_A) += -G M_B / s
 *   node B:  g += +G M_A R_AB / s^3,  phi(R_B) += -G M_A / s
 * Particle pair (a, b), b != a, evaluated once and applied to both (d = r_a - r_b):
 *   g_a += -G m_b d / s^3,  g_b += +G m_a d / s^3,  phi_a += -G m_b / s,  phi_b += -G m_a / s
 * Particle a finally sums, over every node X that contains it, g_X and the first-order
 * potential phi_X(R_X) - g_X . (r_a - R_X).
 *
 * Particles in key order (x, y, z, m); tree from orc_octree (pre-order).  lo, S, bits: the
 * key quantisation (orc_quantise).  Outputs (per particle): g, phi; sg = sum of the norms
 * of the acceleration terms, sp = sum of the magnitudes of the potential terms (the
 * absolute-sum scales), cover = how many other particles reached a through some term
 * (n - 1 when the interactions partition all pairs).  Returns 0, or -1 on a bad tree. */
typedef struct {
    const int32_t* level; const int32_t* leaf; const int64_t* start; const int64_t* count;
    const double *x, *y, *z, *m;
    int64_t* child; int32_t* nch;
    double* mom;          /* 10 per node (orc_moments) */
    int64_t* cell;        /* 3 per node */
    double th4;           /* 4 theta^2 */
    int bits;
    double G, e2;
    double *ng, *nphi, *nsg, *nsp;   /* node accumulators (3, 1, 1, 1) */
    int64_t* ncov;
    double *gx, *gy, *gz, *phi, *sg, *sp;
    int64_t* cover;
} orc_fmm_ctx;

static int orc_fmm_mac(const orc_fmm_ctx* f, int64_t A, int64_t B)
{
    int la = f->level[A], lb = f->level[B];
    int64_t T = ((int64_t)1 << (f->bits - la + 1)) + ((int64_t)1 << (f->bits - lb + 1));
    int64_t D2 = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t ca = (2 * f->cell[3 * A + d] + 1) << (f->bits - la);
        int64_t cb = (2 * f->cell[3 * B + d] + 1) << (f->bits - lb);
        D2 += (ca - cb) * (ca - cb);
    }
    double lhs = 3.0 * (double)(T * T);
    double rhs = f->th4 * (double)D2;
    return lhs < rhs;
}

static void orc_fmm_pair(orc_fmm_ctx* f, int64_t a, int64_t b)
{
    double dx = f->x[a] - f->x[b], dy = f->y[a] - f->y[b], dz = f->z[a] - f->z[b];
    double s = sqrt(dx * dx + dy * dy + dz * dz + f->e2);
    double i1 = 1.0 / s;
    double i3 = i1 * i1 * i1;
    double ka = f->G * f->m[b] * i3, kb = f->G * f->m[a] * i3;
    f->gx[a] -= ka * dx; f->gy[a] -= ka * dy; f->gz[a] -= ka * dz;
    f->gx[b] += kb * dx; f->gy[b] += kb * dy; f->gz[b] += kb * dz;
    f->phi[a] -= f->G * f->m[b] * i1;
    f->phi[b] -= f->G * f->m[a] * i1;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    f->sg[a] += ka * r; f->sg[b] += kb * r;
    f->sp[a] += f->G * f->m[b] * i1; f->sp[b] += f->G * f->m[a] * i1;
    f->cover[a] += 1; f->cover[b] += 1;
}

static void orc_fmm_node_term(orc_fmm_ctx* f, int64_t A, int64_t B)
{
    const double* ma = f->mom + 10 * A;
    const double* mb = f->mom + 10 * B;
    double R[3] = {ma[1] - mb[1], ma[2] - mb[2], ma[3] - mb[3]};
    double s = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2] + f->e2);
    double i1 = 1.0 / s;
    double i3 = i1 * i1 * i1;
    double kA = f->G * mb[0] * i3, kB = f->G * ma[0] * i3;
    double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    for (int d = 0; d < 3; ++d) {
        f->ng[3 * A + d] -= kA * R[d];
        f->ng[3 * B + d] += kB * R[d];
    }
    f->nphi[A] -= f->G * mb[0] * i1;
    f->nphi[B] -= f->G * ma[0] * i1;
    f->nsg[A] += kA * r; f->nsg[B] += kB * r;
    f->nsp[A] += f->G * mb[0] * i1; f->nsp[B] += f->G * ma[0] * i1;
    f->ncov[A] += f->count[B];
    f->ncov[B] += f->count[A];
}

static void orc_fmm_interact(orc_fmm_ctx* f, int64_t A, int64_t B)
{
    if (A == B) {
        if (f->leaf[A]) {
            int64_t s = f->start[A], e = s + f->count[A];
            for (int64_t a = s; a < e; ++a)
                for (int64_t b = a + 1; b < e; ++b) orc_fmm_pair(f, a, b);
        } else {
            const int64_t* c = f->child + 8 * A;
            for (int i = 0; i < f->nch[A]; ++i) orc_fmm_interact(f, c[i], c[i]);
            for (int i = 0; i < f->nch[A]; ++i)
                for (int j = i + 1; j < f->nch[A]; ++j) orc_fmm_interact(f, c[i], c[j]);
        }
        return;
    }
    if (orc_fmm_mac(f, A, B)) {
        orc_fmm_node_term(f, A, B);
        return;
    }
    if (f->leaf[A] && f->leaf[B]) {
        for (int64_t a = f->start[A]; a < f->start[A] + f->count[A]; ++a)
            for (int64_t b = f->start[B]; b < f->start[B] + f->count[B]; ++b) orc_fmm_pair(f, a, b);
        return;
    }
    int split_a = f->level[A] < f->level[B] || (f->level[A] == f->level[B] && f->start[A] < f->start[B]);
    if (split_a ? f->leaf[A] : f->leaf[B]) split_a = !split_a;
    if (split_a) {
        for (int i = 0; i < f->nch[A]; ++i) orc_fmm_interact(f, f->child[8 * A + i], B);
    } else {
        for (int i = 0; i < f->nch[B]; ++i) orc_fmm_interact(f, A, f->child[8 * B + i]);
    }
}

int orc_fmm_gravity(int64_t n, int64_t n_nodes, const int32_t* nlevel, const int32_t* nleaf,
                    const int64_t* nstart, const int64_t* ncount, const double* x, const double* y,
                    const double* z, const double* m, const double* lo3, double S, int bits, double theta,
                    double G, double eps, double* gx, double* gy, double* gz, double* phi, double* sg,
                    double* sp, int64_t* cover)
{
    for (int64_t a = 0; a < n; ++a) { gx[a] = gy[a] = gz[a] = phi[a] = sg[a] = sp[a] = 0.0; cover[a] = 0; }
    if (n_nodes == 0) return 0;
    orc_fmm_ctx f;
    memset(&f, 0, sizeof f);
    f.level = nlevel; f.leaf = nleaf; f.start = nstart; f.count = ncount;
    f.x = x; f.y = y; f.z = z; f.m = m;
    f.bits = bits; f.G = G; f.e2 = eps * eps; f.th4 = 4.0 * (theta * theta);
    f.gx = gx; f.gy = gy; f.gz = gz; f.phi = phi; f.sg = sg; f.sp = sp; f.cover = cover;
    f.child = (int64_t*)malloc(sizeof(int64_t) * 8 * (size_t)n_nodes);
    f.nch = (int32_t*)calloc((size_t)n_nodes, sizeof(int32_t));
    f.mom = (double*)malloc(sizeof(double) * 10 * (size_t)n_nodes);
    f.cell = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)n_nodes);
    f.ng = (double*)calloc(3 * (size_t)n_nodes, sizeof(double));
    f.nphi = (double*)calloc((size_t)n_nodes, sizeof(double));
    f.nsg = (double*)calloc((size_t)n_nodes, sizeof(double));
    f.nsp = (double*)calloc((size_t)n_nodes, sizeof(double));
    f.ncov = (int64_t*)calloc((size_t)n_nodes, sizeof(int64_t));
    int64_t parent_at[23];
    int bad = 0;
    for (int64_t j = 0; j < n_nodes; ++j) {   /* parent = latest node one level up (pre-order) */
        int l = nlevel[j];
        if (l < 0 || l > bits) { bad = 1; break; }
        parent_at[l] = j;
        if (j > 0) {
            int64_t p = parent_at[l - 1];
            if (f.nch[p] >= 8) { bad = 1; break; }
            f.child[8 * p + f.nch[p]++] = j;
        }
        orc_moments(nstart[j], nstart[j] + ncount[j], NULL, x, y, z, m, f.mom + 10 * j);
        const double* c[3] = {x, y, z};
        for (int d = 0; d < 3; ++d)
            f.cell[3 * j + d] = (int64_t)(orc_quantise(c[d][nstart[j]], lo3[d], S, bits) >> (bits - l));
    }
    if (!bad) {
        orc_fmm_interact(&f, 0, 0);
        /* every particle collects the terms of the nodes that contain it */
        int64_t path[23];
        for (int64_t j = 0; j < n_nodes; ++j) {
            path[nlevel[j]] = j;
            if (!nleaf[j]) continue;
            for (int64_t a = nstart[j]; a < nstart[j] + ncount[j]; ++a) {
                const double r[3] = {x[a], y[a], z[a]};
                for (int l = nlevel[0]; l <= nlevel[j]; ++l) {
                    int64_t X = path[l];
                    const double* gX = f.ng + 3 * X;
                    const double* R = f.mom + 10 * X + 1;
                    double lin = gX[0] * (r[0] - R[0]) + gX[1] * (r[1] - R[1]) + gX[2] * (r[2] - R[2]);
                    gx[a] += gX[0]; gy[a] += gX[1]; gz[a] += gX[2];
                    phi[a] += f.nphi[X] - lin;
                    sg[a] += f.nsg[X];
                    sp[a] += f.nsp[X] + fabs(lin);
                    cover[a] += f.ncov[X];
                }
            }
        }
    }
    free(f.child); free(f.nch); free(f.mom); free(f.cell);
    free(f.ng); free(f.nphi); free(f.nsg); free(f.nsp); free(f.ncov);
    return bad ? -1 : 0;
}
