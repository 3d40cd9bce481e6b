/*
 * sph.h -- C ABI of the MI355X (gfx950) SPH + octree hot-path library (libsph_gfx950.so).
 *
 * The library implements, as hand-written HIP kernels, the per-step particle loop of the
 * SPH-plus-tree method of FleCSPH (arXiv:2007.03097): space-filling-curve keys and octree
 * (Sec. 2.1 "Tree topology", Fig. 1), a grouped tree walk that builds per-particle
 * neighbour lists (Sec. 2.1, last paragraph), SPH density and ideal-gas EOS (eq. (7)),
 * momentum and energy equations with artificial viscosity (eqs. (5), (6)), adaptive
 * smoothing length (eq. (9)), octree multipole self-gravity (Sec. 2.2.2, eq. (10)) and a
 * kick-drift-kick leapfrog step.
 *
 * Conventions for every entry point:
 *   - Return value: sph_status; SPH_OK (0) on success, a negative code otherwise.  No C++
 *     exception crosses this interface.  sph_last_error() gives a message.
 *   - Pointers marked "device" are HIP device pointers (e.g. torch .data_ptr()); "host"
 *     pointers are ordinary CPU memory.  The caller owns every particle, output and
 *     workspace buffer; the library owns only its host-side context and HIP graph.
 *   - All particle arrays are float64, structure-of-arrays, in *caller order* (index i is
 *     the caller's particle i, which is also the unique particle ID that breaks key ties,
 *     Sec. 2.1).  Internally the library keeps a Morton-ordered copy in the workspace.
 *   - Calls are asynchronous on the configured stream, except where "synchronous" is
 *     stated.  Conditions found on the device (non-finite input, h <= 0 or m <= 0,
 *     capacity overflow) set a sticky error word that the next synchronous call
 *     (sph_find_neighbors, sph_step, sph_sync) returns.
 *   - Each context may be used by one host thread at a time.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_E_ARG = -1,        /* invalid argument (NULL, size, range); nothing was launched   */
    SPH_E_STATE = -2,      /* call order violated (e.g. forces before density)             */
    SPH_E_NOMEM = -3,      /* workspace missing or too small; host allocation failed       */
    SPH_E_CAPACITY = -4,   /* a fixed capacity was exceeded (neighbours, tree, walk lists) */
    SPH_E_DEVICE = -5,     /* a HIP runtime call failed                                    */
    SPH_E_NONFINITE = -6   /* non-finite x/v/u, or h <= 0, or m <= 0 in the particle data  */
} sph_status;

typedef enum { SPH_FP64 = 0, SPH_FP32C = 1 } sph_precision;

typedef struct sph_ctx sph_ctx;

/* Physics and tuning parameters; fill with sph_config_default() and override. */
typedef struct {
    int32_t precision;   /* SPH_FP64: all pair arithmetic in FP64.  SPH_FP32C: density,
                            force and gravity pair arithmetic in FP32 (SPH positions as FP32
                            offsets from the target group's first particle; quadrupole
                            gravity on FP32 offsets from the group's first target, node-node
                            gravity on FP64 position differences), with Kahan-compensated
                            FP32 sums; neighbour decisions, keys, tree, integration stay
                            FP64/integer.                                                */
    double gamma;        /* ideal-gas adiabatic index (> 1), default 5/3                     */
    double av_alpha;     /* Monaghan viscosity alpha (>= 0), default 1                       */
    double av_beta;      /* Monaghan viscosity beta  (>= 0), default 2                       */
    double av_eps;       /* viscosity regulariser eps in mu = h v.r/(r^2 + eps h^2), 0.01   */
    double h_coeff;      /* C*eta of eq. (9): h = h_coeff (m/rho)^(1/3), default 1.2         */
    int32_t adaptive_h;  /* sph_step: 1 = update h from the density after each step (lagged) */
    double G;            /* gravitational constant; 0 disables gravity in sph_step           */
    double soft_eps;     /* Plummer softening length (>= 0)                                  */
    double theta;        /* opening angle in [0, 1]: a cell whose radius b about its centre of
                            mass (to the farthest corner of its particle box) and distance d
                            from the target group's box satisfy b < theta d is accepted;
                            0 = direct sum                                                 */
    int32_t leaf_size;   /* octree leaf capacity, 1..64 (0 = 16)                             */
    int32_t group_size;  /* target particles per walk group: 8, 16, 32 or 64 (0 = 32)        */
    int32_t nbr_capacity;/* maximum neighbours per particle, 16..4096 (0 = 160)              */
    void* stream;        /* hipStream_t to run on; NULL = the null stream                    */
    int32_t energy_form; /* SPH_ENERGY_THERMAL: u evolves with eq. (5) (default).
                            SPH_ENERGY_THERMOKINETIC: Sec. 2.2.1, eq. (8) -- the total
                            energy e = u + v^2/2 evolves; sph_compute_forces and sph_step's
                            dudt array then carry de/dt (plus v.g when G != 0), and sph_step
                            still takes and returns the thermal u.                      */
    int32_t key_curve;   /* SPH_CURVE_MORTON: Sec. 2.1 / Fig. 1 bit interleave (default).
                            SPH_CURVE_HILBERT: the Hilbert index of the same quantised cell
                            (Skilling's transposition; x, y, z from the high bit of each
                            3-bit digit).  Either way a key's leading 3l bits name its
                            level-l octree cell, so the tree cells, neighbour sets and
                            sums are the same; the sorted order and keys_out differ.    */
    int32_t gravity_scheme; /* SPH_GRAVITY_QUADRUPOLE: particle-cell walk with monopole +
                            quadrupole cells and the opening test above (default).
                            SPH_GRAVITY_FMM: the paper's symmetric node-node scheme (Sec.
                            2.2.2, eq. (10), after Dehnen 2000): node pairs accepted when
                            r_A + r_B < theta |c_A - c_B| (r = sqrt(3)/2 side, c = cell
                            centre) interact through their masses at their centres of mass,
                            first order in the potential (field constant across a node);
                            linear and angular momentum are conserved to rounding.  One set
                            only (n_seg == 1).                                       */
    int32_t waves_per_cu; /* wavefronts per compute unit of the per-group
                            kernels (neighbour walk, density, forces, gravity): their grids
                            hold at most waves_per_cu x 256 wavefronts (256 CUs), fewer when
                            there are fewer groups; 1..32, or 0 (default) for one workgroup
                            per expected group (n over half the group size), as many
                            resident per CU as registers and LDS allow.  Results do not
                            depend on it.                                             */
} sph_config;

/* Values of sph_config.energy_form. */
#define SPH_ENERGY_THERMAL 0
#define SPH_ENERGY_THERMOKINETIC 1
/* Values of sph_config.key_curve. */
#define SPH_CURVE_MORTON 0
#define SPH_CURVE_HILBERT 1
/* Values of sph_config.gravity_scheme. */
#define SPH_GRAVITY_QUADRUPOLE 0
#define SPH_GRAVITY_FMM 1

/* A particle set.  Segments: n_seg > 1 independent sets stored back to back, set s being
 * particles [seg_offsets[s], seg_offsets[s+1]); pairs and tree nodes never cross sets. */
typedef struct {
    int64_t n;                    /* particle count, 0 <= n <= n_capacity                   */
    int32_t n_seg;                /* 1 (seg_offsets may be NULL) or 2..seg_capacity         */
    const int64_t* seg_offsets;   /* host, n_seg + 1 non-decreasing values, 0 .. n          */
    double *x, *y, *z;            /* device: positions                                      */
    double *vx, *vy, *vz;         /* device: velocities                                     */
    double *m, *h, *u;            /* device: masses (> 0), smoothing lengths (> 0),
                                     specific internal energy                               */
    double *ax, *ay, *az, *dudt;  /* device, sph_step only: accelerations and du/dt (de/dt
                                     in the thermokinetic form) of the current state (read
                                     when SPH_STEP_PRIMED, written on return when non-NULL)  */
    const double* seg_dt;         /* host, sph_step only: n_seg step sizes (each > 0), set s
                                     stepping by seg_dt[s]; NULL = every set steps by dt     */
} sph_particles;

/* Flags of sph_step. */
#define SPH_STEP_PRIMED 1u   /* ax..dudt hold the accelerations of the input state          */
#define SPH_STEP_RESUME 2u   /* continue from the state the previous sph_step call left in
                                the workspace; the input arrays are not read                */

/* Fills *cfg with the defaults listed above. */
void sph_config_default(sph_config* cfg);

/* Creates a context for up to n_capacity particles in up to seg_capacity segments
 * (1..512).  Validates cfg (SPH_E_ARG).  n_capacity must keep the octree's node capacity
 * (about 4.4 n_capacity) within 32-bit indices, i.e. n_capacity <= ~4.9e8 (SPH_E_ARG
 * otherwise).  Allocates host memory only. */
sph_status sph_create(const sph_config* cfg, int64_t n_capacity, int32_t seg_capacity, sph_ctx** out);

/* Destroys the context (synchronises its stream, frees the HIP graph). NULL is a no-op. */
sph_status sph_destroy(sph_ctx* ctx);

/* Bytes of device workspace the context needs (depends on capacities and cfg). */
sph_status sph_workspace_size(const sph_ctx* ctx, size_t* bytes);

/* Hands the context a caller-owned device buffer of at least sph_workspace_size() bytes,
 * 256-byte aligned.  The library allocates no device memory of its own. */
sph_status sph_set_workspace(sph_ctx* ctx, void* dev_ptr, size_t bytes);

/* Sec. 2.1: keys, sort and octree.  Computes one key per particle (21 bits per axis inside
 * the set's cubic root cell of side L = largest bounding-box extent, bits interleaved with
 * x lowest, a sentinel bit 63 on top; segmented sets use 18 bits per axis and put the
 * segment number in bits 54..62), sorts by (key, caller index), snapshots the particle
 * data in that order and builds the octree (cells refined while they hold more than
 * leaf_size particles, at most 21 levels).
 *   box_host  host, 6 doubles per segment (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z), or NULL to
 *             use each segment's exact bounding box.
 *   keys_out  device uint64[n] in caller order, or NULL.
 *   order_out device int64[n]: order_out[i] = caller index of the i-th particle in key
 *             order, or NULL. */
sph_status sph_build_tree(sph_ctx* ctx, const sph_particles* ps, const double* box_host,
                          uint64_t* keys_out, int64_t* order_out);

/* The octree of the last sph_build_tree (test and inspection path).  Synchronous.
 * Writes up to capacity nodes (device arrays, any of them NULL to skip):
 *   key    uint64: bit 3*level set (sentinel) followed by the level's 3-bit digits,
 *   level  int32 (0 = root), leaf int32 (1 = leaf), start int64 (first sorted position),
 *   count  int64 (particles in the cell).
 * *n_nodes_host receives the node count; SPH_E_CAPACITY if it exceeds capacity. */
sph_status sph_tree_nodes(sph_ctx* ctx, int64_t capacity, uint64_t* key, int32_t* level, int32_t* leaf,
                          int64_t* start, int64_t* count, int64_t* n_nodes_host);

/* Sec. 2.1 (group traversal that builds a neighbour list per particle): neighbours of a
 * are the b (self included, same segment) with |r_a - r_b| < h_a + h_b, decided in FP64
 * exactly as fl(fl(fl(dx dx) + fl(dy dy)) + fl(dz dz)) < fl(t t), t = fl(h_a + h_b).
 * Builds the lists for the last tree, then exports them as CSR in caller order, each list
 * sorted by ascending caller index.  Synchronous.
 *   offsets_out device int64[n + 1];  idx_out device int32[capacity].
 *   *total_host receives the number of entries; SPH_E_CAPACITY (nothing written to
 *   idx_out) if it exceeds capacity.  SPH_E_CAPACITY also when a particle has more than
 *   nbr_capacity neighbours, or when the source union of a walk group (the particles that
 *   are a neighbour of at least one of its group_size targets) exceeds 65,536 particles:
 *   the device lists hold 16-bit indices into that union.  Either output may be NULL to
 *   only count.  With all three of offsets_out, idx_out and total_host NULL the call only
 *   (re)builds the device lists, asynchronously (used to time the list kernel). */
sph_status sph_find_neighbors(sph_ctx* ctx, int64_t* offsets_out, int32_t* idx_out, int64_t capacity,
                              int64_t* total_host);

/* Eq. (7) density with W_ab = W(r_ab, h_ab), h_ab = (h_a + h_b)/2, M4 cubic spline of
 * support 2h, self term included; ideal-gas EOS P = (gamma-1) rho u, c = sqrt(gamma P/rho);
 * eq. (9) h_next = h_coeff (m/rho)^(1/3).  Builds neighbour lists if needed.
 * Outputs: device double[n] in caller order; any may be NULL (the values stay in the
 * workspace for sph_compute_forces either way). */
sph_status sph_compute_density(sph_ctx* ctx, double* rho, double* P, double* cs, double* h_next);

/* Eqs. (6) and (5) with g = 0: dv_a/dt = -sum_b m_b ((P_a/rho_a^2 + P_b/rho_b^2) + Pi_ab)
 * grad_a W_ab and du_a/dt = sum_b m_b (P_a/rho_a^2 + Pi_ab/2) v_ab . grad_a W_ab, with the
 * Monaghan viscosity Pi_ab = (-alpha cbar mu + beta mu^2)/rhobar for v_ab . r_ab < 0,
 * mu = h_ab v_ab . r_ab / (r^2 + eps h_ab^2).  rho, P, cs: device double[n] in caller order,
 * or all NULL to use the values of the last sph_compute_density (SPH_E_STATE if none
 * since the last sph_build_tree, or if the last sph_compute_forces was given values).
 * With energy_form = SPH_ENERGY_THERMOKINETIC, dudt receives eq. (8) instead:
 * de_a/dt = -sum_b m_b (P_a v_b/rho_a^2 + P_b v_a/rho_b^2 + (v_a + v_b)/2 Pi_ab) . grad_a W_ab.
 * Outputs: device double[n] in caller order; any may be NULL (not copied out). */
sph_status sph_compute_forces(sph_ctx* ctx, const double* rho, const double* P, const double* cs,
                              double* ax, double* ay, double* az, double* dudt);

/* Sec. 2.2.2, eq. (10): self-gravity on the last tree.  Cells accepted by the opening test
 * (see sph_config.theta) act through monopole + quadrupole moments about their centre of
 * mass, with Plummer softening; other leaves by direct softened sums (self excluded).
 * With gravity_scheme = SPH_GRAVITY_FMM: the symmetric node-node scheme instead (see
 * sph_config.gravity_scheme); particle pairs of unaccepted leaf pairs are summed directly,
 * and phi is the first-order potential.  SPH_E_ARG if the last tree holds several sets.
 * With G == 0 (gravity off) the outputs are filled with zeros: such a context builds its trees
 * without node masses and moments, which only gravity reads.
 * Outputs: device double[n] in caller order; any may be NULL (not copied out). */
sph_status sph_compute_gravity(sph_ctx* ctx, double* gx, double* gy, double* gz, double* phi);

/* Work of the last particle-cell gravity pass (Sec. 2.2.2; the tree code's cost, Sec. 3.4),
 * from sph_compute_gravity or the last step that evaluated gravity: *cells_host = cell terms
 * evaluated (each accepted cell times the targets of its group), *pairs_host = particle-
 * particle terms (each unaccepted leaf's particles times the group's targets, the targets'
 * own pairs taken out).  At theta = 0 these are 0 and n (n - 1) for one set.  Synchronises the
 * stream.  SPH_E_STATE when gravity is off or uses the node-node scheme (not counted). */
sph_status sph_gravity_counts(sph_ctx* ctx, int64_t* cells_host, int64_t* pairs_host);

/* nsteps kick-drift-kick leapfrog steps of size dt (> 0; per set when ps->seg_dt is given):
 *   v' = v + dt/2 a;  u' = u + dt/2 du;  x += dt v';  predictors v^ = v' + dt/2 a, u^ = u' + dt/2 du;
 *   rebuild keys, tree and neighbours; density, EOS(u^), forces with v^ (+ gravity if G != 0);
 *   v = v' + dt/2 a_new;  u = u' + dt/2 du_new;  adaptive_h: h = h_coeff (m/rho)^(1/3).
 * Thermokinetic form: the same scheme integrates e = u + v^2/2 with de/dt (eq. (8), plus
 * v^.g with gravity) in place of u; the EOS takes u^ = e^ - |v^|^2/2, and the returned u is
 * e - |v|^2/2.
 * Without SPH_STEP_PRIMED the accelerations of the input state are computed first (and,
 * with adaptive_h, h is reset from that density).  The state stays on the device in key
 * order between steps; on return x, v, u, h (and ax..dudt when given) are written back in
 * caller order.  Synchronous.
 *   diag_host host double[10] or NULL: Px, Py, Pz, Lx, Ly, Lz, E_kin, E_th, E_grav of the
 *   final state (FP64 sums in a fixed order; E_grav = sum m phi / 2 with the last gravity
 *   pass's potential), then the smallest time-step bound over all sets (see sph_timestep;
 *   NaN when no density pass has run on the state, i.e. nsteps = 0 with SPH_STEP_PRIMED). */
sph_status sph_step(sph_ctx* ctx, sph_particles* ps, double dt, int32_t nsteps, uint32_t flags,
                    double* diag_host);

/* Time-step bound of the state the last sph_step left on the device (the step criterion of
 * the configurations: a Courant-type h/c limit and, with self-gravity, the free-fall limit of
 * the softening length): per set s, bound_host[s] = min over its particles of
 * min(h_a/c_a, sqrt(soft_eps/|a_a|)), the second term only when G != 0 and soft_eps > 0 and
 * |a_a| > 0.  h is the current smoothing length, c the sound speed of the last density pass
 * (at the step's predicted state), a the last accelerations (gravity included).  The caller
 * scales it by its Courant factor (0.25 in the configurations).  An empty set gives +inf.
 *   bound_host host double[n_seg].  Synchronous.
 * SPH_E_STATE without a previous sph_step, or when no density pass has run on the state. */
sph_status sph_timestep(sph_ctx* ctx, double* bound_host);

/* Keys and key order of the set the context holds (test and inspection path): after
 * sph_build_tree, its keys and order; after sph_step, the keys of the step's last key sort
 * (computed at the returned positions with each set's box of those positions) and the order
 * of the resident state.  Synchronous.
 *   keys_out  device uint64[n] in caller order, or NULL.
 *   order_out device int64[n]: caller index of the i-th particle in key order, or NULL.
 * SPH_E_STATE without a previous sph_build_tree or sph_step. */
sph_status sph_key_order(sph_ctx* ctx, uint64_t* keys_out, int64_t* order_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sph_step with the context's kernels
 * working in the library's own static device scratch of SPH_NOALLOC_MAX_BYTES bytes instead
 * of the caller's workspace.  The call allocates nothing (no hipMalloc, hipFree, graph
 * objects or library allocations; launches are eager on cfg.stream) and needs no
 * sph_set_workspace.  Same arguments, results and synchronisation as sph_step.
 *   - SPH_E_CAPACITY if the context's workspace size (sph_workspace_size: it grows with
 *     n_capacity, seg_capacity and nbr_capacity) exceeds the scratch; about 27,000
 *     particles fit with nbr_capacity 160, 36,000 with 64.
 *   - Every call on one GPU shares that GPU's scratch, which keeps the last call's
 *     contents: calls that overlap on one GPU (other threads, other streams) race, and
 *     SPH_STEP_RESUME is accepted only when no other call used the scratch since this
 *     context's last one (SPH_E_STATE otherwise).  The scratch state is separate from the
 *     workspace state: sph_step, sph_timestep and sph_key_order see only the latter.
 *   - The scratch stays allocated on each GPU the library has run on until the process
 *     ends. */
#define SPH_NOALLOC_MAX_BYTES (64u << 20)
sph_status sph_step_noalloc(sph_ctx* ctx, sph_particles* ps, double dt, int32_t nsteps, uint32_t flags,
                            double* diag_host);

/* Times sph_step over candidate leaf_size x group_size settings on ps (which it leaves
 * unchanged), then over waves_per_cu for the fastest pair, keeps the fastest in the context
 * and records "key": [leaf_size, group_size, waves_per_cu] in a JSON cache file
 * (cache_json_path may be NULL).  A cached entry is used as it is; an entry with only
 * [leaf_size, group_size] keeps those and has its waves_per_cu searched and recorded.
 * Synchronous. */
sph_status sph_autotune(sph_ctx* ctx, const sph_particles* ps, double dt, const char* cache_json_path);

/* Current tuning parameters of the context; any pointer may be NULL. */
sph_status sph_get_tuning(const sph_ctx* ctx, int32_t* leaf_size, int32_t* group_size, int32_t* waves_per_cu);

/* Waits for the context's stream and returns (and clears) the sticky device error. */
sph_status sph_sync(sph_ctx* ctx);

/* Message for the last failed call on ctx (static text for ctx == NULL). */
const char* sph_last_error(const sph_ctx* ctx);

/* Device peak probe, for reading the kernels' arithmetic rates against a measured ceiling (no
 * context, no SPH state).  Launches asynchronously on `stream` (a hipStream_t; NULL = the
 * default stream) n_threads / 256 workgroups of 256 threads; each thread runs 8 independent
 * fused-multiply-add chains of `iters` links in FP64 (kind 0) or unpacked FP32 (kind 1) and
 * stores their sum to out_dev[thread].  One call performs 16 * iters * n_threads flops; timing
 * it with events gives the sustained vector FMA rate.
 *   out_dev  device double[n_threads], caller-owned, overwritten.
 * SPH_E_ARG: kind not 0 or 1, out_dev NULL, n_threads <= 0 or not a multiple of 256, iters <= 0.
 * SPH_E_DEVICE: the launch failed. */
sph_status sph_peak_probe(int32_t kind, double* out_dev, int64_t n_threads, int32_t iters, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
