// C ABI of the gfx950 SPH + octree library (declarations and contracts in include/sph.h).
//
// Host-side responsibilities: argument validation, carving the caller's workspace into the
// device arrays, the host-built chunk and segment tables, launch sequencing on the caller's
// stream, capture of one leapfrog step per buffer parity into HIP graphs, the sticky device
// error word, and the autotuner.  No device memory is allocated here.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "../../include/sph.h"

namespace {

constexpr int CHUNK = 1024;

struct Tables {
    int64_t n = -1;
    int n_seg = 0;
    int gsz = 0;
    std::vector<int64_t> seg;  // offsets
    int version = 0;           // identifies the device tables; never reused within a context
};

}  // namespace

// The device memory one context works in, with the state that lives there.  A context has
// two: the caller's workspace (sph_set_workspace) and the library's static scratch
// (sph_step_noalloc); the active one sits in the context's own fields.
struct Binding {
    char* ws = nullptr;
    size_t ws_bytes = 0;
    DevPtrs d[2]{};
    Dims dm{};
    Tables tab;
    bool tree_ok = false, lists_ok = false, dens_ok = false, resident_ok = false, cs_ok = false;
    int parity = 0;
};

struct sph_ctx {
    sph_config cfg{};
    int64_t n_cap = 0;
    int seg_cap = 1;
    int leaf_min = 16;        // smallest leaf size the workspace is sized for
    int leaf_size = 16;
    int group_size = 32;
    int waves = 0;            // waves per CU of the per-group kernels (0 = one workgroup per group)
    int nbr_cap = 160;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    DevPtrs d[2]{};           // pointer sets: d[p] has the resident state in buffer set p
    Dims dm{};
    Tables tab;
    int tab_gen = 0;          // last table version handed out (only ever increases)
    std::vector<double> seg_dt;  // step size per segment of the current sph_step call
    bool cs_ok = false;       // the resident sound speeds belong to the resident state
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    bool tree_ok = false, lists_ok = false, dens_ok = false, resident_ok = false;
    int parity = 0;
    // step graphs [k][p]: from buffer set p, k = 0 the first step of a run, k = 1 a later one
    hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int64_t g_n = -1;
    int g_leaf = 0, g_gsz = 0, g_waves = -1, g_tabv = -1;
    bool use_graph = true;
    Binding alt;              // the binding not in use (the scratch one outside sph_step_noalloc)
    unsigned scratch_gen = 0; // the device scratch generation this context's scratch state has
    std::string err;
};

static const char* k_null_ctx_msg = "sph: NULL context";

static sph_status fail(sph_ctx* c, sph_status st, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return st;
}

#define HIPCHK(ctx, call)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return fail((ctx), SPH_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------------------
// workspace layout

static int64_t node_cap_for(int64_t n, int leaf) { return 2 * n + 21 * n / (leaf + 1) + 256; }

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

static size_t layout(const sph_ctx* c, char* base, DevPtrs* out) {
    const size_t N = (size_t)std::max<int64_t>(c->n_cap, 1);
    const size_t S = (size_t)c->seg_cap;
    const size_t NC = (size_t)node_cap_for((int64_t)N, c->leaf_min);
    const size_t GC = N + 8;                             // a group holds at least one particle
    const size_t NBR = N * (size_t)c->nbr_cap + 64;      // group blocks tile n * nbr_cap words
    const size_t CH = N / CHUNK + S + 1;
    const size_t RSB = (N + 2047) / 2048;
    const size_t SCB = (std::max(N + 1, 256 * RSB) + 2047) / 2048 + 16;
    const size_t LST = (NC + 2047) / 2048 + 1;
    Carver cv{base};
    DevPtrs d{};
    d.ctl = cv.take<DevCtl>(1);
    d.key_a = cv.take<u64>(N);
    d.key_b = cv.take<u64>(N);
    d.val_a = cv.take<u32>(N);
    d.val_b = cv.take<u32>(N);
    d.rs_hist = cv.take<u32>(256 * RSB);
    d.rs_dtot = cv.take<u32>(256);
    d.scan_tmp = cv.take<u64>(SCB);
    double** f1[] = {&d.x, &d.y, &d.z, &d.vx, &d.vy, &d.vz, &d.m, &d.h, &d.u, &d.vpx, &d.vpy, &d.vpz, &d.up,
                     &d.ax, &d.ay, &d.az, &d.du, &d.rho, &d.P, &d.cs, &d.hnext, &d.gx, &d.gy, &d.gz, &d.phi,
                     &d.x2, &d.y2, &d.z2, &d.vx2, &d.vy2, &d.vz2, &d.m2, &d.h2, &d.u2, &d.vpx2, &d.vpy2, &d.vpz2,
                     &d.up2};
    for (double** p : f1) *p = cv.take<double>(N);
    d.id = cv.take<u32>(N);
    d.id2 = cv.take<u32>(N);
    d.pos4 = cv.take<double4>(N);
    d.vel4 = cv.take<double4>(N);
    d.thr4 = cv.take<double4>(N);
    d.thrf = cv.take<float4>(N);
    d.lcp = cv.take<signed char>(N + 1);
    d.lvl = cv.take<unsigned char>(N);
    d.scan_in = cv.take<u64>(N + 1);
    d.scan_out = cv.take<u64>(N + 1);
    d.leaf_start = cv.take<int>(N + 1);
    d.leaf_pre = cv.take<int>(N);
    d.pre_level = cv.take<unsigned char>(NC);
    d.pre_leaf = cv.take<unsigned char>(NC);
    d.pre_start = cv.take<int>(NC);
    d.pre_to_bfs = cv.take<int>(NC);
    d.bfs_to_pre = cv.take<int>(NC);
    d.lsort_hist = cv.take<int>(24 * LST);
    d.topo = cv.take<int4>(NC);
    d.parent = cv.take<int>(NC);
    d.counter = cv.take<int>(NC);
    d.range = cv.take<int2>(NC);
    d.nbox_lo = cv.take<double4>(NC);
    d.nbox_hi = cv.take<double4>(NC);
    d.mom0 = cv.take<double4>(NC);
    d.mom1 = cv.take<double4>(NC);
    d.mom2 = cv.take<double4>(NC);
    d.group = cv.take<int4>(GC);
    d.gflag = cv.take<u32>(N + 1);
    d.gscan = cv.take<u32>(N + 1);
    d.gsize = cv.take<u32>(N + 1);
    d.nbr = cv.take<u16>(NBR);
    d.nbr_cnt = cv.take<int>(N);
    d.nbr_base = cv.take<int>(N);
    d.uni = cv.take<int>(NBR);
    d.ucnt = cv.take<int>(GC);
    d.chunk = cv.take<int4>(CH);
    d.seg_root_rank = cv.take<int>(S);
    d.diag_part = cv.take<double>(16 * 256);
    d.csr_tmp = cv.take<int64_t>(N + 1);
    if (out) *out = d;
    return cv.off + 256;
}

static DevPtrs swapped(const DevPtrs& a) {
    DevPtrs b = a;
    std::swap(b.x, b.x2); std::swap(b.y, b.y2); std::swap(b.z, b.z2);
    std::swap(b.vx, b.vx2); std::swap(b.vy, b.vy2); std::swap(b.vz, b.vz2);
    std::swap(b.m, b.m2); std::swap(b.h, b.h2); std::swap(b.u, b.u2);
    std::swap(b.vpx, b.vpx2); std::swap(b.vpy, b.vpy2); std::swap(b.vpz, b.vpz2); std::swap(b.up, b.up2);
    std::swap(b.id, b.id2);
    return b;
}

// ---------------------------------------------------------------------------------------
// validation helpers

static sph_status check_config(sph_ctx* c, const sph_config* f) {
    if (!f) return fail(c, SPH_E_ARG, "config is NULL");
    if (f->precision != SPH_FP64 && f->precision != SPH_FP32C) return fail(c, SPH_E_ARG, "precision must be 0 or 1");
    if (!(f->gamma > 1.0) || !std::isfinite(f->gamma)) return fail(c, SPH_E_ARG, "gamma must be > 1");
    if (!(f->av_alpha >= 0.0) || !(f->av_beta >= 0.0) || !(f->av_eps >= 0.0))
        return fail(c, SPH_E_ARG, "viscosity parameters must be >= 0");
    if (!(f->h_coeff > 0.0)) return fail(c, SPH_E_ARG, "h_coeff must be > 0");
    if (!(f->theta >= 0.0 && f->theta <= 1.0)) return fail(c, SPH_E_ARG, "theta must be in [0, 1]");
    if (!(f->soft_eps >= 0.0) || !std::isfinite(f->soft_eps)) return fail(c, SPH_E_ARG, "soft_eps must be >= 0");
    if (!std::isfinite(f->G)) return fail(c, SPH_E_ARG, "G must be finite");
    const int L = f->leaf_size ? f->leaf_size : 16;
    if (L < 1 || L > 64) return fail(c, SPH_E_ARG, "leaf_size must be in 1..64");
    const int g = f->group_size ? f->group_size : 32;
    if (g != 8 && g != 16 && g != 32 && g != 64) return fail(c, SPH_E_ARG, "group_size must be 8, 16, 32 or 64");
    const int k = f->nbr_capacity ? f->nbr_capacity : 160;
    if (k < 16 || k > 4096) return fail(c, SPH_E_ARG, "nbr_capacity must be in 16..4096");
    if (f->energy_form != SPH_ENERGY_THERMAL && f->energy_form != SPH_ENERGY_THERMOKINETIC)
        return fail(c, SPH_E_ARG, "energy_form must be 0 or 1");
    if (f->key_curve != SPH_CURVE_MORTON && f->key_curve != SPH_CURVE_HILBERT)
        return fail(c, SPH_E_ARG, "key_curve must be 0 or 1");
    if (f->gravity_scheme != SPH_GRAVITY_QUADRUPOLE && f->gravity_scheme != SPH_GRAVITY_FMM)
        return fail(c, SPH_E_ARG, "gravity_scheme must be 0 or 1");
    if (f->waves_per_cu < 0 || f->waves_per_cu > 32) return fail(c, SPH_E_ARG, "waves_per_cu must be in 0..32");
    return SPH_OK;
}

static sph_status check_particles(sph_ctx* c, const sph_particles* p) {
    if (!p) return fail(c, SPH_E_ARG, "particles is NULL");
    if (p->n < 0 || p->n > c->n_cap) return fail(c, SPH_E_ARG, "n = %lld outside 0..%lld", (long long)p->n, (long long)c->n_cap);
    if (p->n_seg < 1 || p->n_seg > c->seg_cap) return fail(c, SPH_E_ARG, "n_seg = %d outside 1..%d", p->n_seg, c->seg_cap);
    if (p->n_seg > 1 && !p->seg_offsets) return fail(c, SPH_E_ARG, "seg_offsets required when n_seg > 1");
    if (p->seg_offsets) {
        if (p->seg_offsets[0] != 0 || p->seg_offsets[p->n_seg] != p->n)
            return fail(c, SPH_E_ARG, "seg_offsets must start at 0 and end at n");
        for (int s = 0; s < p->n_seg; ++s)
            if (p->seg_offsets[s + 1] < p->seg_offsets[s]) return fail(c, SPH_E_ARG, "seg_offsets not monotone");
    }
    if (p->n > 0 && (!p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->m || !p->h || !p->u))
        return fail(c, SPH_E_ARG, "a particle array is NULL");
    if (!c->ws) return fail(c, SPH_E_NOMEM, "no workspace set");
    return SPH_OK;
}

// Host tables for the current set: chunks (bounding box / keys) and segment ranks.  The
// target groups are built on the device with the tree.
static sph_status prepare(sph_ctx* c, const sph_particles* p) {
    const int n_seg = p->n_seg;
    std::vector<int64_t> seg(n_seg + 1);
    if (p->seg_offsets) for (int s = 0; s <= n_seg; ++s) seg[s] = p->seg_offsets[s];
    else { seg[0] = 0; seg[1] = p->n; }
    Dims& dm = c->dm;
    dm.n = (int)p->n;
    dm.n_seg = n_seg;
    dm.batched = n_seg > 1;
    dm.leaf_size = c->leaf_size;
    dm.group_size = c->group_size;
    dm.nbr_cap = c->nbr_cap;
    dm.node_cap = (int)node_cap_for(c->n_cap > 0 ? c->n_cap : 1, c->leaf_min);
    dm.min_level = dm.batched ? 3 : 0;
    dm.curve = c->cfg.key_curve;
    dm.mass_moments = c->cfg.G != 0.0;
    const bool same = c->tab.n == p->n && c->tab.n_seg == n_seg && c->tab.seg == seg;
    std::vector<int4> chunks;
    std::vector<int> rank(n_seg, 0);
    int r = 0;
    for (int s = 0; s < n_seg; ++s) {
        rank[s] = r;
        if (seg[s + 1] > seg[s]) ++r;
        for (int64_t b = seg[s]; b < seg[s + 1]; b += CHUNK)
            chunks.push_back(make_int4((int)b, (int)std::min<int64_t>(seg[s + 1], b + CHUNK), s, b == seg[s]));
    }
    dm.n_chunks = (int)chunks.size();
    {   // grids of the per-group kernels: multiples of 8 (one share per XCD), one workgroup per
        // expected group (groups average over half of group_size); the kernels loop over any
        // groups beyond that.  Groups differ widely in cost, and the hardware dispatcher, which
        // starts a workgroup wherever one ends, balances them better than a resident-sized grid
        // with a fixed share per workgroup.  With waves_per_cu, at most that many wavefronts
        // per CU (one-wave and four-wave workgroups).
        const int64_t est = p->n / std::max(1, c->group_size / 2) + 8;
        const int64_t units = (est + 7) / 8;
        int64_t u1 = units, u4 = units;
        if (c->waves > 0) {
            u1 = std::min<int64_t>(units, (int64_t)c->waves * 256 / 8);
            u4 = std::min<int64_t>(units, std::max<int64_t>(1, (int64_t)c->waves * 256 / 4 / 8));
        }
        dm.group_grid = (int)(8 * u1);
        dm.pair_grid = (int)(8 * u4);
    }
    if (!same) {
        if (!chunks.empty())
            HIPCHK(c, hipMemcpyAsync(c->d[0].chunk, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice,
                                     c->stream));
        HIPCHK(c, hipMemcpyAsync(c->d[0].seg_root_rank, rank.data(), rank.size() * sizeof(int), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));  // host vectors go out of scope
        c->tab.n = p->n;
        c->tab.n_seg = n_seg;
        c->tab.seg = seg;
        c->tab.version = ++c->tab_gen;
    }
    return SPH_OK;
}

static sph_status read_err(sph_ctx* c) {
    u32 e = 0;
    HIPCHK(c, hipMemcpyAsync(&e, &c->d[0].ctl->err, sizeof e, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!e) return SPH_OK;
    const u32 zero = 0;
    HIPCHK(c, hipMemcpyAsync(&c->d[0].ctl->err, &zero, sizeof zero, hipMemcpyHostToDevice, c->stream));
    int nmax = 0;
    HIPCHK(c, hipMemcpyAsync(&nmax, &c->d[0].ctl->nbr_max, sizeof nmax, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (e & (ERR_NONFINITE | ERR_NONPOSITIVE))
        return fail(c, SPH_E_NONFINITE, "device (error word 0x%x): %s%s", e, (e & ERR_NONFINITE) ? "non-finite x/v/u " : "",
                    (e & ERR_NONPOSITIVE) ? "h <= 0 or m <= 0" : "");
    if (e & ERR_NBR_CAP) return fail(c, SPH_E_CAPACITY, "device: neighbour list overflow (%d > nbr_capacity %d)", nmax, c->nbr_cap);
    if (e & ERR_WALK_STACK) return fail(c, SPH_E_CAPACITY, "device: tree-walk stack or candidate list overflow");
    if (e & ERR_UNION_CAP)
        return fail(c, SPH_E_CAPACITY, "device: a walk group's source union exceeds %d particles", UNION_MAX);
    if (e & ERR_NODE_CAP) return fail(c, SPH_E_CAPACITY, "device: octree node capacity exceeded");
    if (e & ERR_GRAV_LIST) return fail(c, SPH_E_CAPACITY, "device: gravity walk stack overflow");
    return fail(c, SPH_E_DEVICE, "device error word 0x%x", e);
}

// Exchanges the active binding (the context's fields) with c->alt.
static void swap_binding(sph_ctx* c) {
    Binding& b = c->alt;
    std::swap(c->ws, b.ws);
    std::swap(c->ws_bytes, b.ws_bytes);
    std::swap(c->d[0], b.d[0]);
    std::swap(c->d[1], b.d[1]);
    std::swap(c->dm, b.dm);
    std::swap(c->tab, b.tab);
    std::swap(c->tree_ok, b.tree_ok);
    std::swap(c->lists_ok, b.lists_ok);
    std::swap(c->dens_ok, b.dens_ok);
    std::swap(c->resident_ok, b.resident_ok);
    std::swap(c->cs_ok, b.cs_ok);
    std::swap(c->parity, b.parity);
}

// Forgets the captured step graphs (they hold workspace pointers and table sizes by value).
static void drop_graphs(sph_ctx* c) {
    for (int k = 0; k < 2; ++k)
        for (int p = 0; p < 2; ++p) {
            if (c->gexec[k][p]) { (void)hipGraphExecDestroy(c->gexec[k][p]); c->gexec[k][p] = nullptr; }
            if (c->graph[k][p]) { (void)hipGraphDestroy(c->graph[k][p]); c->graph[k][p] = nullptr; }
        }
    c->g_tabv = -1;
    c->g_n = -1;
}

// keys (caller order) -> sort -> key-ordered snapshot in buffer set 0 -> octree
static sph_status build_from_caller(sph_ctx* c, const sph_particles* p, const double* box_host, uint64_t* keys_out,
                                    int64_t* order_out) {
    sph_status st = prepare(c, p);
    if (st != SPH_OK) return st;
    c->parity = 0;
    c->tree_ok = c->lists_ok = c->dens_ok = c->resident_ok = c->cs_ok = false;
    const DevPtrs& d = c->d[0];
    const Dims& dm = c->dm;
    if (dm.n == 0) {
        c->tree_ok = true;
        return SPH_OK;
    }
    if (box_host) {
        HIPCHK(c, hipMemcpyAsync(d.ctl->box, box_host, sizeof(double) * 6 * dm.n_seg, hipMemcpyHostToDevice, c->stream));
        launch_set_box(c->stream, d, dm, 1);
    } else {
        launch_bbox(c->stream, d, dm, p->x, p->y, p->z, nullptr);
        launch_set_box(c->stream, d, dm, 0);
    }
    launch_keys(c->stream, d, dm, p->x, p->y, p->z, p->vx, p->vy, p->vz, p->m, p->h, p->u, (u64*)keys_out, 1);
    radix_sort(c->stream, d, dm.n);
    launch_gather_input(c->stream, d, dm, p->x, p->y, p->z, p->vx, p->vy, p->vz, p->m, p->h, p->u, order_out);
    build_octree(c->stream, d, dm);
    HIPCHK(c, hipGetLastError());
    c->tree_ok = true;
    return SPH_OK;
}

static sph_status ensure_lists(sph_ctx* c) {
    if (!c->tree_ok) return fail(c, SPH_E_STATE, "sph_build_tree has not been called");
    if (!c->lists_ok) {
        launch_nbr_lists(c->stream, c->d[c->parity], c->dm);
        HIPCHK(c, hipGetLastError());
        c->lists_ok = true;
    }
    return SPH_OK;
}

// Self-gravity of the resident state with the configured scheme; accumulate adds it to
// a (and v.g to du when thermo), else it goes to g and phi.
static void gravity_pass(sph_ctx* c, hipStream_t s, const DevPtrs& d, int accumulate, int thermo) {
    const int fp32c = c->cfg.precision == SPH_FP32C;
    if (c->cfg.gravity_scheme == SPH_GRAVITY_FMM)
        launch_fmm(s, d, c->dm, fp32c, c->cfg.G, c->cfg.soft_eps, c->cfg.theta, accumulate, thermo);
    else
        launch_gravity(s, d, c->dm, fp32c, c->cfg.G, c->cfg.soft_eps, c->cfg.theta, accumulate, thermo);
}

// ---------------------------------------------------------------------------------------
extern "C" {

void sph_config_default(sph_config* f) {
    if (!f) return;
    memset(f, 0, sizeof *f);
    f->precision = SPH_FP64;
    f->gamma = 5.0 / 3.0;
    f->av_alpha = 1.0;
    f->av_beta = 2.0;
    f->av_eps = 0.01;
    f->h_coeff = 1.2;
    f->adaptive_h = 0;
    f->G = 0.0;
    f->soft_eps = 0.0;
    f->theta = 0.5;
    f->leaf_size = 16;
    f->group_size = 32;
    f->nbr_capacity = 160;
    f->energy_form = SPH_ENERGY_THERMAL;
    f->key_curve = SPH_CURVE_MORTON;
    f->gravity_scheme = SPH_GRAVITY_QUADRUPOLE;
    f->waves_per_cu = 0;
    f->stream = nullptr;
}

sph_status sph_create(const sph_config* cfg, int64_t n_capacity, int32_t seg_capacity, sph_ctx** out) {
    if (!out) return SPH_E_ARG;
    *out = nullptr;
    if (n_capacity < 0 || n_capacity > (1ll << 30)) return SPH_E_ARG;
    if (seg_capacity < 1 || seg_capacity > 512) return SPH_E_ARG;
    sph_ctx* c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_E_NOMEM;
    sph_status st = check_config(c, cfg);
    if (st != SPH_OK) {
        delete c;
        return st;
    }
    c->cfg = *cfg;
    c->n_cap = n_capacity;
    c->seg_cap = seg_capacity;
    c->leaf_size = cfg->leaf_size ? cfg->leaf_size : 16;
    c->leaf_min = std::min(c->leaf_size, 8);
    if (node_cap_for(std::max<int64_t>(n_capacity, 1), c->leaf_min) >= (int64_t)INT32_MAX) {
        delete c;  // node indices are 32-bit
        return SPH_E_ARG;
    }
    c->group_size = cfg->group_size ? cfg->group_size : 32;
    c->waves = cfg->waves_per_cu;
    c->nbr_cap = cfg->nbr_capacity ? cfg->nbr_capacity : 160;
    c->stream = (hipStream_t)cfg->stream;
    const char* ng = getenv("SPH_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    *out = c;
    return SPH_OK;
}

sph_status sph_destroy(sph_ctx* c) {
    if (!c) return SPH_OK;
    if (c->ws) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return SPH_OK;
}

sph_status sph_workspace_size(const sph_ctx* c, size_t* bytes) {
    if (!c || !bytes) return SPH_E_ARG;
    *bytes = layout(c, nullptr, nullptr);
    return SPH_OK;
}

sph_status sph_set_workspace(sph_ctx* c, void* ptr, size_t bytes) {
    if (!c) return SPH_E_ARG;
    if (!ptr) return fail(c, SPH_E_ARG, "workspace pointer is NULL");
    if (((uintptr_t)ptr) & 255) return fail(c, SPH_E_ARG, "workspace must be 256-byte aligned");
    const size_t need = layout(c, nullptr, nullptr);
    if (bytes < need) return fail(c, SPH_E_NOMEM, "workspace too small: %zu < %zu bytes", bytes, need);
    c->ws = (char*)ptr;
    c->ws_bytes = bytes;
    layout(c, c->ws, &c->d[0]);
    c->d[1] = swapped(c->d[0]);
    DevCtl zero;
    memset(&zero, 0, sizeof zero);
    HIPCHK(c, hipMemcpyAsync(c->d[0].ctl, &zero, sizeof zero, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->tab = Tables();
    drop_graphs(c);
    c->tree_ok = c->lists_ok = c->dens_ok = c->resident_ok = c->cs_ok = false;
    return SPH_OK;
}

sph_status sph_build_tree(sph_ctx* c, const sph_particles* p, const double* box_host, uint64_t* keys_out,
                          int64_t* order_out) {
    if (!c) return SPH_E_ARG;
    sph_status st = check_particles(c, p);
    if (st != SPH_OK) return st;
    return build_from_caller(c, p, box_host, keys_out, order_out);
}

sph_status sph_tree_nodes(sph_ctx* c, int64_t capacity, uint64_t* key, int32_t* level, int32_t* leaf, int64_t* start,
                          int64_t* count, int64_t* n_nodes_host) {
    if (!c || !n_nodes_host) return SPH_E_ARG;
    if (!c->tree_ok) return fail(c, SPH_E_STATE, "sph_build_tree has not been called");
    int nn = 0;
    if (c->dm.n > 0) {
        HIPCHK(c, hipMemcpyAsync(&nn, &c->d[0].ctl->n_nodes, sizeof nn, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    *n_nodes_host = nn;
    if (nn > capacity) return fail(c, SPH_E_CAPACITY, "tree has %d nodes > capacity %lld", nn, (long long)capacity);
    if (nn > 0) launch_tree_export(c->stream, c->d[c->parity], c->dm, (u64*)key, level, leaf, start, count);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return read_err(c);
}

sph_status sph_find_neighbors(sph_ctx* c, int64_t* offsets_out, int32_t* idx_out, int64_t capacity,
                              int64_t* total_host) {
    if (!c) return SPH_E_ARG;
    if (!offsets_out && !idx_out && !total_host) {  // rebuild the lists only (asynchronous)
        if (!c->tree_ok) return fail(c, SPH_E_STATE, "sph_build_tree has not been called");
        c->lists_ok = false;
        return ensure_lists(c);
    }
    sph_status st = ensure_lists(c);
    if (st != SPH_OK) return st;
    const DevPtrs& d = c->d[c->parity];
    const int n = c->dm.n;
    int64_t total = 0;
    if (n > 0) {
        launch_csr_count(c->stream, d, c->dm, d.csr_tmp);
        scan_i64_inplace(c->stream, d.csr_tmp, n, d.scan_tmp);
        HIPCHK(c, hipMemcpyAsync(&total, d.csr_tmp + n, sizeof total, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    st = read_err(c);
    if (st != SPH_OK) return st;
    if (total_host) *total_host = total;
    if (offsets_out) {
        if (n > 0)
            HIPCHK(c, hipMemcpyAsync(offsets_out, d.csr_tmp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, c->stream));
        else {
            const int64_t z = 0;
            HIPCHK(c, hipMemcpyAsync(offsets_out, &z, sizeof z, hipMemcpyHostToDevice, c->stream));
        }
    }
    if (idx_out) {
        if (total > capacity) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            return fail(c, SPH_E_CAPACITY, "%lld neighbour entries > capacity %lld", (long long)total, (long long)capacity);
        }
        if (n > 0) launch_csr_fill(c->stream, d, c->dm, d.csr_tmp, idx_out);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SPH_OK;
}

sph_status sph_compute_density(sph_ctx* c, double* rho, double* P, double* cs, double* h_next) {
    if (!c) return SPH_E_ARG;
    sph_status st = ensure_lists(c);
    if (st != SPH_OK) return st;
    const DevPtrs& d = c->d[c->parity];
    const int n = c->dm.n;
    launch_density(c->stream, d, c->dm, c->cfg.precision == SPH_FP32C, c->cfg.gamma, c->cfg.h_coeff, d.u, 0);
    launch_scatter_caller(c->stream, d, n, d.rho, rho);
    launch_scatter_caller(c->stream, d, n, d.P, P);
    launch_scatter_caller(c->stream, d, n, d.cs, cs);
    launch_scatter_caller(c->stream, d, n, d.hnext, h_next);
    HIPCHK(c, hipGetLastError());
    c->dens_ok = true;
    return SPH_OK;
}

sph_status sph_compute_forces(sph_ctx* c, const double* rho, const double* P, const double* cs, double* ax, double* ay,
                              double* az, double* dudt) {
    if (!c) return SPH_E_ARG;
    const int n = c->dm.n;
    const int given = (rho != nullptr) + (P != nullptr) + (cs != nullptr);
    if (given != 0 && given != 3) return fail(c, SPH_E_ARG, "rho, P, cs must be all given or all NULL");
    sph_status st = ensure_lists(c);
    if (st != SPH_OK) return st;
    const DevPtrs& d = c->d[c->parity];
    if (given == 3) {
        launch_thermo_from_caller(c->stream, d, c->dm, rho, P, cs);
        c->dens_ok = false;
    } else if (!c->dens_ok) {
        return fail(c, SPH_E_STATE, "sph_compute_density has not been called");
    }
    launch_forces(c->stream, d, c->dm, c->cfg.precision == SPH_FP32C, c->cfg.av_alpha, c->cfg.av_beta, c->cfg.av_eps,
                  c->cfg.energy_form == SPH_ENERGY_THERMOKINETIC);
    launch_scatter_caller(c->stream, d, n, d.ax, ax);
    launch_scatter_caller(c->stream, d, n, d.ay, ay);
    launch_scatter_caller(c->stream, d, n, d.az, az);
    launch_scatter_caller(c->stream, d, n, d.du, dudt);
    HIPCHK(c, hipGetLastError());
    return SPH_OK;
}

sph_status sph_compute_gravity(sph_ctx* c, double* gx, double* gy, double* gz, double* phi) {
    if (!c) return SPH_E_ARG;
    const int n = c->dm.n;
    if (!c->tree_ok) return fail(c, SPH_E_STATE, "sph_build_tree has not been called");
    if (c->cfg.gravity_scheme == SPH_GRAVITY_FMM && c->dm.batched)
        return fail(c, SPH_E_ARG, "gravity_scheme SPH_GRAVITY_FMM needs a single set (n_seg == 1)");
    if (c->cfg.G == 0.0) {  // no gravity: the tree carries no mass moments
        for (double* o : {gx, gy, gz, phi}) launch_fill_zero(c->stream, n, o);
        HIPCHK(c, hipGetLastError());
        return SPH_OK;
    }
    const DevPtrs& d = c->d[c->parity];
    launch_fill_i32(c->stream, &d.ctl->skip_phi, 0, 1);  // this pass returns the potential
    gravity_pass(c, c->stream, d, 0, 0);
    launch_scatter_caller(c->stream, d, n, d.gx, gx);
    launch_scatter_caller(c->stream, d, n, d.gy, gy);
    launch_scatter_caller(c->stream, d, n, d.gz, gz);
    launch_scatter_caller(c->stream, d, n, d.phi, phi);
    HIPCHK(c, hipGetLastError());
    return SPH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// leapfrog driver

// Accelerations of the resident state in buffer set p (tree already built).
// u_eos holds e = u + v^2/2 when kin (thermokinetic steps), the thermal u otherwise.
static void accel_pass(sph_ctx* c, hipStream_t s, const DevPtrs& d, const double* u_eos, int kin) {
    const int fp32c = c->cfg.precision == SPH_FP32C;
    const int thermo = c->cfg.energy_form == SPH_ENERGY_THERMOKINETIC;
    launch_nbr_lists(s, d, c->dm);
    launch_density(s, d, c->dm, fp32c, c->cfg.gamma, c->cfg.h_coeff, u_eos, kin);
    launch_forces(s, d, c->dm, fp32c, c->cfg.av_alpha, c->cfg.av_beta, c->cfg.av_eps, thermo);
    if (c->cfg.G != 0.0) gravity_pass(c, s, d, 1, thermo);
}

// One KDK step from buffer set p into buffer set 1 - p, without its closing half kick: a run
// of steps applies each closing kick at the start of the next step (the kick-drift's PRE form,
// the same accelerations and roundings) and the last one after the run (close_run).
static void step_launches(sph_ctx* c, hipStream_t s, int p, bool later) {
    const DevPtrs& a = c->d[p];
    const DevPtrs& b = c->d[1 - p];
    const int n = c->dm.n;
    if (!later) launch_box_init(s, a, c->dm);  // later steps: the previous permute reset the box
    launch_kick_drift(s, a, c->dm, later, c->cfg.adaptive_h);  // also merges the new box
    launch_step_keys(s, a, c->dm);        // also derives L and S
    radix_sort(s, a, n);
    launch_step_permute(s, a, n);         // also writes the pair records
    build_octree(s, b, c->dm);
    accel_pass(c, s, b, b.up, c->cfg.energy_form == SPH_ENERGY_THERMOKINETIC);
}

// The last step's closing half kick (and lagged h update), on the resident state.
static void close_run(sph_ctx* c, hipStream_t s) { launch_kick(s, c->d[c->parity], c->dm, c->cfg.adaptive_h); }

// The kernels read each segment's step size from the control block, so a change of dt
// needs no new graph.
static sph_status run_steps(sph_ctx* c, int nsteps) {
    if (nsteps <= 0 || c->dm.n == 0) return SPH_OK;
    HIPCHK(c, hipMemcpyAsync(c->d[0].ctl->seg_dt, c->seg_dt.data(), sizeof(double) * c->seg_dt.size(),
                             hipMemcpyHostToDevice, c->stream));
    const bool regraph = c->g_n != c->dm.n || c->g_leaf != c->leaf_size || c->g_gsz != c->group_size ||
                         c->g_waves != c->waves || c->g_tabv != c->tab.version;
    // Only the last step's potential is read (by the diagnostics of the final state): the
    // gravity passes skip it before that.  Set on the stream between the steps, so the
    // captured step graphs are the same for every step.
    int* skip_phi = &c->d[0].ctl->skip_phi;
    const bool thin = c->cfg.G != 0.0 && nsteps > 1;
    auto phi_flag = [&](int k) {
        if (thin && k == 0) launch_fill_i32(c->stream, skip_phi, 1, 1);
        if (thin && k == nsteps - 1) launch_fill_i32(c->stream, skip_phi, 0, 1);
    };
    if (!c->use_graph) {
        for (int k = 0; k < nsteps; ++k) {
            phi_flag(k);
            step_launches(c, c->stream, c->parity, k > 0);
            c->parity ^= 1;
        }
        close_run(c, c->stream);
        HIPCHK(c, hipGetLastError());
        return SPH_OK;
    }
    if (regraph || !c->gexec[0][0] || !c->gexec[0][1] || !c->gexec[1][0] || !c->gexec[1][1]) {
        if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        drop_graphs(c);
        for (int k = 0; k < 2; ++k)
            for (int p = 0; p < 2; ++p) {
                HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                step_launches(c, c->cap_stream, p, k > 0);
                HIPCHK(c, hipStreamEndCapture(c->cap_stream, &c->graph[k][p]));
                HIPCHK(c, hipGraphInstantiate(&c->gexec[k][p], c->graph[k][p], nullptr, nullptr, 0));
            }
        c->g_n = c->dm.n;
        c->g_tabv = c->tab.version;
        c->g_leaf = c->leaf_size;
        c->g_gsz = c->group_size;
        c->g_waves = c->waves;
    }
    for (int k = 0; k < nsteps; ++k) {
        phi_flag(k);
        HIPCHK(c, hipGraphLaunch(c->gexec[k > 0][c->parity], c->stream));
        c->parity ^= 1;
    }
    close_run(c, c->stream);
    HIPCHK(c, hipGetLastError());
    return SPH_OK;
}

static sph_status step_impl(sph_ctx* c, sph_particles* p, double dt, int32_t nsteps, uint32_t flags, double* diag,
                            bool write_back) {
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, SPH_E_ARG, "dt must be > 0");
    if (nsteps < 0) return fail(c, SPH_E_ARG, "nsteps must be >= 0");
    if (p && p->seg_dt) {
        const int ns = (flags & SPH_STEP_RESUME) ? c->dm.n_seg : p->n_seg;
        if ((flags & SPH_STEP_RESUME) && p->n_seg != ns)
            return fail(c, SPH_E_ARG, "SPH_STEP_RESUME with a different number of sets");
        if (ns < 1 || ns > c->seg_cap) return fail(c, SPH_E_ARG, "n_seg = %d outside 1..%d", ns, c->seg_cap);
        for (int s = 0; s < ns; ++s)
            if (!(p->seg_dt[s] > 0.0) || !std::isfinite(p->seg_dt[s]))
                return fail(c, SPH_E_ARG, "seg_dt[%d] must be > 0", s);
    }
    sph_status st;
    if (flags & SPH_STEP_RESUME) {
        if (!c->resident_ok) return fail(c, SPH_E_STATE, "SPH_STEP_RESUME without a previous sph_step");
        if (!c->ws) return fail(c, SPH_E_NOMEM, "no workspace set");
        if (p && p->n != c->dm.n) return fail(c, SPH_E_ARG, "SPH_STEP_RESUME with a different particle count");
    } else {
        st = check_particles(c, p);
        if (st != SPH_OK) return st;
        if (c->cfg.G != 0.0 && c->cfg.gravity_scheme == SPH_GRAVITY_FMM && p->n_seg > 1)
            return fail(c, SPH_E_ARG, "gravity_scheme SPH_GRAVITY_FMM needs a single set (n_seg == 1)");
        if ((flags & SPH_STEP_PRIMED) && p->n > 0 && (!p->ax || !p->ay || !p->az || !p->dudt))
            return fail(c, SPH_E_ARG, "SPH_STEP_PRIMED needs ax, ay, az and dudt");
        st = build_from_caller(c, p, nullptr, nullptr, nullptr);
        if (st != SPH_OK) return st;
        const DevPtrs& d = c->d[0];
        const int n = c->dm.n;
        launch_fill_i32(c->stream, &d.ctl->skip_phi, 0, 1);  // the primed state's potential too
        if (n > 0) {
            if (flags & SPH_STEP_PRIMED) {
                launch_load_accel(c->stream, d, n, p->ax, p->ay, p->az, p->dudt);
            } else {
                accel_pass(c, c->stream, d, d.u, 0);
                if (c->cfg.adaptive_h) launch_set_hnext(c->stream, d, n);
                c->cs_ok = true;
            }
            if (c->cfg.energy_form == SPH_ENERGY_THERMOKINETIC) launch_add_kinetic(c->stream, d, n);
        }
        HIPCHK(c, hipGetLastError());
        c->resident_ok = true;
    }
    c->tree_ok = c->lists_ok = c->dens_ok = false;
    c->seg_dt.assign(c->dm.n_seg, dt);
    if (p && p->seg_dt) c->seg_dt.assign(p->seg_dt, p->seg_dt + c->dm.n_seg);
    st = run_steps(c, nsteps);
    if (st != SPH_OK) return st;
    if (nsteps > 0 && c->dm.n > 0) c->cs_ok = true;
    const DevPtrs& d = c->d[c->parity];
    const int n = c->dm.n;
    if (diag) {
        launch_diag(c->stream, d, c->dm, c->cfg.G != 0.0, c->cfg.energy_form == SPH_ENERGY_THERMOKINETIC,
                    c->cfg.G != 0.0 ? c->cfg.soft_eps : 0.0);
        HIPCHK(c, hipMemcpyAsync(diag, d.ctl->diag, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    if (write_back && p && p->x && n > 0)
        launch_write_back(c->stream, d, n, p->x, p->y, p->z, p->vx, p->vy, p->vz, p->h, p->u, p->ax, p->ay, p->az,
                          p->dudt, c->cfg.energy_form == SPH_ENERGY_THERMOKINETIC);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (diag && !c->cs_ok) diag[9] = NAN;  // no density pass on this state yet
    return read_err(c);
}

extern "C" {

sph_status sph_timestep(sph_ctx* c, double* bound_host) {
    if (!c || !bound_host) return SPH_E_ARG;
    if (!c->resident_ok) return fail(c, SPH_E_STATE, "sph_timestep needs the state of a previous sph_step");
    if (!c->cs_ok) return fail(c, SPH_E_STATE, "sph_timestep: no density pass on the resident state yet");
    const int ns = c->dm.n_seg;
    if (c->dm.n == 0) {
        for (int s = 0; s < ns; ++s) bound_host[s] = INFINITY;
        return SPH_OK;
    }
    const DevPtrs& d = c->d[c->parity];
    launch_dt_bound(c->stream, d, c->dm, c->cfg.G != 0.0 ? c->cfg.soft_eps : 0.0);
    std::vector<u64> enc(ns);
    HIPCHK(c, hipMemcpyAsync(enc.data(), d.ctl->dtb_enc, sizeof(u64) * ns, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < ns; ++s) {  // the ordered-integer encoding of k_dt_bound, inverted
        const u64 e = enc[s];
        const u64 b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
        double v;
        memcpy(&v, &b, sizeof v);
        bound_host[s] = v;
    }
    return read_err(c);
}

sph_status sph_gravity_counts(sph_ctx* c, int64_t* cells_host, int64_t* pairs_host) {
    if (!c || !cells_host || !pairs_host) return SPH_E_ARG;
    if (c->cfg.G == 0.0 || c->cfg.gravity_scheme == SPH_GRAVITY_FMM)
        return fail(c, SPH_E_STATE, "sph_gravity_counts: no particle-cell gravity pass in this context");
    u64 slots[GRAV_SLOTS][16];
    HIPCHK(c, hipMemcpyAsync(slots, c->d[0].ctl->grav_cnt, sizeof slots, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    u64 v[2] = {0, 0};
    for (int s = 0; s < GRAV_SLOTS; ++s) {
        v[0] += slots[s][0];
        v[1] += slots[s][1];
    }
    *cells_host = (int64_t)v[0];
    *pairs_host = (int64_t)v[1] - (v[1] > 0 ? (int64_t)c->dm.n : 0);  // the targets' own pairs
    return read_err(c);
}

sph_status sph_key_order(sph_ctx* c, uint64_t* keys_out, int64_t* order_out) {
    if (!c) return SPH_E_ARG;
    if (!c->tree_ok && !c->resident_ok)
        return fail(c, SPH_E_STATE, "sph_key_order needs a previous sph_build_tree or sph_step");
    launch_resident_export(c->stream, c->d[c->parity], c->dm.n, (u64*)keys_out, order_out);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return read_err(c);
}

sph_status sph_step(sph_ctx* c, sph_particles* p, double dt, int32_t nsteps, uint32_t flags, double* diag_host) {
    if (!c) return SPH_E_ARG;
    return step_impl(c, p, dt, nsteps, flags, diag_host, true);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Allocation-free stepping: the context works in a file-scope device array instead of the
// caller's workspace.  In host code `scratch` names a host-side stand-in; its device address
// on each GPU comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_MAX_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
unsigned g_scratch_gen[MAX_DEVICES] = {};  // calls made on each device's scratch
}  // namespace

__global__ void k_zero_words(u32* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

extern "C" {

sph_status sph_step_noalloc(sph_ctx* c, sph_particles* p, double dt, int32_t nsteps, uint32_t flags,
                            double* diag_host) {
    if (!c) return SPH_E_ARG;
    const size_t need = layout(c, nullptr, nullptr);
    if (need > (size_t)SPH_NOALLOC_MAX_BYTES)
        return fail(c, SPH_E_CAPACITY, "sph_step_noalloc: the context needs %zu bytes of device memory, more than the "
                    "%zu-byte scratch (lower n_capacity, seg_capacity or nbr_capacity)", need,
                    (size_t)SPH_NOALLOC_MAX_BYTES);
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(c, SPH_E_DEVICE, "sph_step_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {  // once per device, with that device current
        void* ptr = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255)) return fail(c, SPH_E_DEVICE, "sph_step_noalloc: bad scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    char* base = (char*)g_scratch_ptr[dev];
    if (flags & SPH_STEP_RESUME) {  // the scratch must still hold this context's state
        if (c->alt.ws != base || c->scratch_gen != g_scratch_gen[dev] || !c->alt.resident_ok)
            return fail(c, SPH_E_STATE, "SPH_STEP_RESUME: the scratch no longer holds this context's state");
    }
    if (c->alt.ws != base) {  // first use on this device: bind the scratch, control block cleared
        c->alt = Binding();
        c->alt.ws = base;
        c->alt.ws_bytes = SPH_NOALLOC_MAX_BYTES;
        layout(c, base, &c->alt.d[0]);
        c->alt.d[1] = swapped(c->alt.d[0]);
    }
    if (!(flags & SPH_STEP_RESUME)) {
        c->alt.tab = Tables();  // another context may have changed the tables in the scratch
        const int words = (int)(sizeof(DevCtl) / sizeof(u32));
        hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, c->stream, (u32*)c->alt.d[0].ctl,
                           words);
        HIPCHK(c, hipGetLastError());
    }
    g_scratch_gen[dev]++;
    c->scratch_gen = g_scratch_gen[dev];
    swap_binding(c);
    const bool graph = c->use_graph;
    c->use_graph = false;  // eager launches: no graph objects are created or destroyed
    const sph_status st = step_impl(c, p, dt, nsteps, flags, diag_host, true);
    c->use_graph = graph;
    swap_binding(c);
    return st;
}

sph_status sph_get_tuning(const sph_ctx* c, int32_t* leaf_size, int32_t* group_size, int32_t* waves_per_cu) {
    if (!c) return SPH_E_ARG;
    if (leaf_size) *leaf_size = c->leaf_size;
    if (group_size) *group_size = c->group_size;
    if (waves_per_cu) *waves_per_cu = c->waves;
    return SPH_OK;
}

sph_status sph_autotune(sph_ctx* c, const sph_particles* p, double dt, const char* cache) {
    if (!c) return SPH_E_ARG;
    sph_status st = check_particles(c, p);
    if (st != SPH_OK) return st;
    char keybuf[160];
    snprintf(keybuf, sizeof keybuf, "n%lld_s%d_p%d_g%d_a%d%s", (long long)p->n, p->n_seg, c->cfg.precision,
             c->cfg.G != 0.0, c->cfg.adaptive_h,
             c->cfg.G != 0.0 && c->cfg.gravity_scheme == SPH_GRAVITY_FMM ? "_fmm" : "");
    const std::string key(keybuf);
    std::string body;  // the cache file (tiny JSON object of "key": [leaf, group, waves])
    if (cache) {
        std::ifstream f(cache);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            body = ss.str();
        }
    }
    const std::string qkey = "\"" + key + "\"";
    const size_t at = body.find(qkey);
    int cL = 0, cG = 0, cW = -1;
    bool cached = false;
    if (at != std::string::npos && body.find('[', at) != std::string::npos) {
        const int got = sscanf(body.c_str() + body.find('[', at), "[%d, %d, %d]", &cL, &cG, &cW);
        cached = got >= 2 && cL >= c->leaf_min && cL <= 64 && (cG == 8 || cG == 16 || cG == 32 || cG == 64);
        if (got < 3 || cW < 0 || cW > 32) cW = -1;
    }
    if (cached && cW >= 0) {
        c->leaf_size = cL;
        c->group_size = cG;
        c->waves = cW;
        return SPH_OK;
    }
    sph_particles q = *p;
    q.ax = q.ay = q.az = q.dudt = nullptr;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // milliseconds of 3 steps (after a load, prime, warm-up and capture), or a negative value
    auto time_steps = [&](int L, int G, int W) -> double {
        c->leaf_size = L;
        c->group_size = G;
        c->waves = W;
        if (step_impl(c, &q, dt, 1, 0, nullptr, false) != SPH_OK) return -1.0;
        if (hipEventRecord(e0, c->stream) != hipSuccess) return -1.0;
        if (step_impl(c, &q, dt, 3, SPH_STEP_RESUME, nullptr, false) != SPH_OK) return -1.0;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        return ms;
    };
    double best = 1e300;
    int bL = c->leaf_size, bG = c->group_size;
    if (cached) {
        bL = cL;
        bG = cG;
        const double ms = time_steps(bL, bG, 0);
        if (ms >= 0.0) best = ms;
    } else {
        // the node-node gravity favours larger leaves (its particle sums fill more lanes)
        const bool fmm = c->cfg.G != 0.0 && c->cfg.gravity_scheme == SPH_GRAVITY_FMM;
        const std::vector<int> leaves =
            fmm ? std::vector<int>{16, 24, 32, 48, 64} : std::vector<int>{8, 12, 16, 24, 32};
        const int groups[] = {16, 32, 64};
        for (int L : leaves) {
            if (L < c->leaf_min) continue;
            for (int G : groups) {
                const double ms = time_steps(L, G, 0);
                if (ms >= 0.0 && ms < best) {
                    best = ms;
                    bL = L;
                    bG = G;
                }
            }
        }
    }
    // waves per CU for the chosen sizes; a cap must win by more than 1% over the default
    int bW = 0;
    if (best < 1e300) {
        double bw = best;
        for (int W : {4, 8, 12, 16, 24}) {
            const double ms = time_steps(bL, bG, W);
            if (ms >= 0.0 && ms < 0.99 * bw) {
                bw = ms;
                bW = W;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->leaf_size = bL;
    c->group_size = bG;
    c->waves = bW;
    c->resident_ok = c->cs_ok = false;
    c->tab = Tables();
    drop_graphs(c);
    if (cache && best < 1e300) {
        char entry[256];
        snprintf(entry, sizeof entry, "%s: [%d, %d, %d]", qkey.c_str(), bL, bG, bW);
        if (at != std::string::npos) {  // replace the entry of this key
            const size_t end = body.find(']', at);
            body = body.substr(0, at) + entry + (end == std::string::npos ? std::string() : body.substr(end + 1));
        } else {
            const size_t close = body.rfind('}');
            if (close == std::string::npos || body.find('"') == std::string::npos)
                body = std::string("{\n  ") + entry + "\n}\n";
            else
                body = body.substr(0, close) + ",\n  " + entry + "\n}\n";
        }
        std::ofstream o(cache);
        o << body;
    }
    return best < 1e300 ? SPH_OK : fail(c, SPH_E_DEVICE, "autotune: no configuration ran");
}

sph_status sph_sync(sph_ctx* c) {
    if (!c) return SPH_E_ARG;
    if (!c->ws) return SPH_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return read_err(c);
}

const char* sph_last_error(const sph_ctx* c) {
    if (!c) return k_null_ctx_msg;
    return c->err.c_str();
}

}  // extern "C"
