// Host side of the C ABI declared in include/lbm.h: validation, workspace
// layout, kernel launches and error reporting.  No exception crosses the ABI.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                        \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t elem_bytes(int prec) {
    switch (prec) {
        case LB_F64:
            return 8;
        case LB_F32:
            return 4;
        case LB_F16DEV:
        case LB_BF16DEV:
            return 2;
        default:
            return 0;
    }
}

int64_t nodes(const lb_params *p) { return int64_t(p->nx) * p->ny * p->nz; }

// Workspace layout (all offsets 256-byte aligned):
//   mat      : N bytes, working material map with flag bits
//   ledger   : max_tiles * 2 doubles, per-xy-tile reservoir ledger; with the
//              evaporation sink max_tiles * nz more pairs, one per work-group
//              (xy tile, z chunk) of the step
//   heights  : with the sink, [2][nz][ny*nx] int32 liquid-node counts per
//              column and z chunk (read by one step, written by the other)
//   status   : 256 bytes (status word)
//   partials : OBS_BLOCKS * OBS_FIELDS doubles
//   result   : 256 bytes
//   psi      : 16 x 2 doubles, ghost pseudo-densities per material id
//   carry    : 2 doubles, ledger folded out of the tile slots on tile changes
//   rods     : n_rods x ROD_STRIDE doubles
//   rodid    : N int16, rod id per node (-1 none); newid: N int32
//   rodsum   : 8 doubles (solid ledger, rod momentum)
//   rodpart  : 3 x n_rods x rod_nblk x ROD_PART doubles, per-block partial sums
//   shell    : n_rods x rod_shell_cap int32 surface lists; shell_cnt: n_rods int32
//   nbr      : n_rods x ROD_NBR int16 neighbour lists; nbr_cnt: n_rods int32
//
// Capacity of a rod's surface list (nodes within R + 3/2 of the axis): the
// unit cells centred on those nodes are disjoint and lie within
// R + 3/2 + sqrt(3)/2 of the axis segment, so their number is at most that
// capsule's volume.  Rounded up to whole 256-thread work-groups.
static int rod_shell_cap(const lb_params &p) {
    const double pi = 3.14159265358979323846;
    const double half = 0.5 * p.rod_length - p.rod_radius;
    const double rr = p.rod_radius + 1.5 + 0.5 * std::sqrt(3.0);
    const double vol = pi * rr * rr * 2.0 * half + 4.0 / 3.0 * pi * rr * rr * rr;
    return int((std::ceil(vol) + 255.0) / 256.0) * 256;
}
static int rod_nblk(const lb_params &p) { return rod_shell_cap(p) / 256; }

// Observable scratch: droplet column scan, then deposit binning and graph.
struct ObsLayout {
    size_t col_h, col_wet, line_x, line_y, out, bins, sval, dep_out, ens_acc, ens_out, labels, graph, map, probe_xyz,
        probe_p, total;
};
static ObsLayout obs_layout(const lb_params *p) {
    ObsLayout l{};
    const size_t ncol = size_t(p->nx) * p->ny, nr = size_t(std::max(p->n_rods, 0));
    size_t o = 0;
    l.col_h = o;
    o = align256(o + ncol * sizeof(double));
    l.col_wet = o;
    o = align256(o + ncol * sizeof(int));
    l.line_x = o;
    o = align256(o + size_t(p->nx) * sizeof(double));
    l.line_y = o;
    o = align256(o + size_t(p->ny) * sizeof(double));
    l.out = o;
    o = align256(o + 16 * sizeof(double));
    l.bins = o;
    o = align256(o + nr * 4 * DEP_NB * sizeof(int16_t));
    l.sval = o;
    o = align256(o + nr * sizeof(double));
    l.dep_out = o;
    o = align256(o + 6 * DEP_MAXBIN * sizeof(double));
    l.ens_acc = o;
    o = align256(o + 8 * DEP_MAXBIN * sizeof(double));
    l.ens_out = o;
    o = align256(o + 6 * DEP_MAXBIN * sizeof(double));
    l.labels = o;
    o = align256(o + nr * sizeof(int32_t));
    l.graph = o;
    o = align256(o + 4 * sizeof(int32_t));
    l.map = o;
    o = align256(o + ncol * sizeof(int32_t));
    l.probe_xyz = o;
    o = align256(o + 3 * PROBE_MAX * sizeof(int32_t));
    l.probe_p = o;
    o = align256(o + PROBE_MAX * sizeof(double));
    l.total = o;
    return l;
}
static size_t obs_bytes(const lb_params *p) { return obs_layout(p).total; }

struct WsLayout {
    size_t mat, ledger, heights, status, partials, result, psi, carry, rods, rodid, newid, rodsum, rodpart, shell, shell_cnt,
        nbr, nbr_cnt, rodargs, rho, cg, fil, fil_sten, fil_nbr, fil_cnt, fil_grid, fil_claim, fil_led, obs, total;
    int max_tiles;
    int nslots;  // ledger slot pairs
};

int fil_beads(const lb_params *p) { return p->n_fil > 0 && p->fil_beads > 0 ? p->n_fil * p->fil_beads : 0; }

WsLayout ws_layout(const lb_params *p) {
    WsLayout w{};
    const int64_t n = nodes(p);
    w.max_tiles = tiles_xy(p->nx, p->ny, 4);
    size_t o = 0;
    w.mat = o;
    o = align256(o + size_t(n));
    w.ledger = o;
    w.nslots = w.max_tiles * (p->sink_on ? 1 + p->nz : 1);
    o = align256(o + size_t(w.nslots) * 2 * sizeof(double));
    w.heights = o;
    o = align256(o + (p->sink_on ? 2 * size_t(n) * sizeof(int32_t) : 0));
    w.status = o;
    o = align256(o + 256);
    w.partials = o;
    o = align256(o + size_t(OBS_BLOCKS) * OBS_FIELDS * sizeof(double));
    w.result = o;
    o = align256(o + 256);
    w.psi = o;
    o = align256(o + 32 * sizeof(double));
    w.carry = o;
    o = align256(o + 2 * sizeof(double));
    w.rods = o;
    o = align256(o + size_t(std::max(p->n_rods, 0)) * ROD_STRIDE * sizeof(double));
    const size_t idb = p->n_rods > 0 ? size_t(n) * sizeof(int16_t) : 0;
    w.rodid = o;
    o = align256(o + idb);
    w.newid = o;
    o = align256(o + 2 * idb);  // int32
    w.rodsum = o;
    o = align256(o + 8 * sizeof(double));
    w.rodpart = o;
    const size_t nr = size_t(std::max(p->n_rods, 0));
    const bool rods = nr > 0;
    o = align256(o + (rods ? 3 * nr * rod_nblk(*p) * ROD_PART * sizeof(double) : 0));
    w.shell = o;
    o = align256(o + (rods ? nr * rod_shell_cap(*p) * sizeof(int) : 0));
    w.shell_cnt = o;
    o = align256(o + nr * sizeof(int));
    w.nbr = o;
    o = align256(o + nr * ROD_NBR * sizeof(int16_t));
    w.nbr_cnt = o;
    o = align256(o + nr * sizeof(int));
    w.rodargs = o;
    o = align256(o + (rods ? 2 * sizeof(RodArgs) : 0));
    // fluid densities of the current state in compute precision, written by
    // the fluid step for the rod passes
    w.rho = o;
    const bool dens = rods || fil_beads(p) > 0;
    o = align256(o + (dens ? 2 * size_t(lb_pop_stride(p)) * (p->prec == LB_F64 ? 8 : 4) : 0));
    // filaments: bead records, stencils, partner lists, the fixed-point
    // momentum grid [3][fs] and its claim flags [fs]
    const size_t nb = size_t(fil_beads(p));
    const bool fil = nb > 0;
    w.fil = o;
    o = align256(o + nb * FIL_STRIDE * sizeof(double));
    w.fil_sten = o;
    o = align256(o + nb * 8 * sizeof(int));
    w.fil_nbr = o;
    o = align256(o + nb * FIL_NBR * sizeof(int));
    w.fil_cnt = o;
    o = align256(o + nb * sizeof(int));
    w.fil_grid = o;
    o = align256(o + (fil ? 3 * size_t(lb_pop_stride(p)) * sizeof(long long) : 0));
    w.fil_claim = o;
    o = align256(o + (fil ? size_t(lb_pop_stride(p)) * sizeof(int) : 0));
    w.fil_led = o;
    o = align256(o + (fil ? 2 * sizeof(long long) : 0));
    // colour-gradient step: colour [fs] and normal [4][fs] in compute precision
    w.cg = o;
    o = align256(o + (p->model == LB_MODEL_CG ? 5 * size_t(lb_pop_stride(p)) * (p->prec == LB_F64 ? 8 : 4) : 0));
    w.obs = o;
    o = align256(o + obs_bytes(p));
    w.total = o;
    return w;
}

bool tile_ok(int ty, int rp, bool tau1) {
    const bool ok = (ty == 4 && rp == 1) || (ty == 8 && (rp == 1 || rp == 2)) || (ty == 16 && rp == 2);
    return ok && (tau1 || rp == 1);
}

int validate(const lb_params *p) {
    if (!p) return fail(LB_EINVAL, "null params");
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return fail(LB_EINVAL, "lattice must be at least 3 nodes per direction");
    if (nodes(p) > (int64_t(1) << 31) / 2) return fail(LB_EINVAL, "lattice too large for one context");
    if (elem_bytes(p->prec) == 0) return fail(LB_ENOTSUP, "unknown precision %d", p->prec);
    // the step kernel addresses each component's 19 arrays through one buffer
    // resource with 32-bit byte offsets
    const uint64_t comp_bytes = uint64_t(Q) * uint64_t(((nodes(p) + 255) / 256) * 256 + 64) * elem_bytes(p->prec);
    if (comp_bytes > 0xFFFFFFFFull) return fail(LB_EINVAL, "lattice too large: one component exceeds 4 GiB");
    for (int k = 0; k < 2; ++k)
        if (!(p->tau[k] > 0.5)) return fail(LB_EINVAL, "tau[%d] = %g must exceed 1/2", k, p->tau[k]);
    if (!isfinite(p->G)) return fail(LB_EINVAL, "G not finite");
    const int ty = p->tile_y ? p->tile_y : 8;
    const int rp = p->rows_per_thread;
    const int rp1 = p->rows_per_thread ? p->rows_per_thread : 1;
    const bool tau1 = p->tau[0] == 1.0 && p->tau[1] == 1.0;
    if (!tile_ok(ty, rp1, true)) return fail(LB_EINVAL, "unsupported tile %d x %d rows per thread", ty, rp);
    if (!tau1 && rp1 != 1) return fail(LB_ENOTSUP, "tau != 1 needs rows_per_thread = 1 (populations stay in registers)");
    if (p->evap_on && p->nz < 4) return fail(LB_EINVAL, "evaporation needs nz >= 4");
    if (p->sink_on) {
        // FP32 storage, or FP64 with tau = 1 (the FP64 step with the sink runs
        // only the instantiations checked against the oracle)
        const bool t1 = p->tau[0] == 1.0 && p->tau[1] == 1.0;
        if (!(p->prec == LB_F32 || (p->prec == LB_F64 && t1)))
            return fail(LB_ENOTSUP, "the evaporation sink runs with FP32 storage, or FP64 with tau = 1");
        if (!(p->sink_J0 >= 0.0) || !isfinite(p->sink_J0) || !(p->sink_K >= 0.0) || !isfinite(p->sink_K) ||
            !(p->sink_h0 > 0.0) || !isfinite(p->sink_h0))
            return fail(LB_EINVAL, "sink needs J0 >= 0, K >= 0 and h0 > 0 (finite)");
    }
    if (p->model != LB_MODEL_SC && p->model != LB_MODEL_CG) return fail(LB_EINVAL, "unknown fluid model %d", p->model);
    if (p->model == LB_MODEL_CG) {
        if (p->prec != LB_F64 && p->prec != LB_F32)
            return fail(LB_ENOTSUP, "the colour-gradient step runs with FP64 or FP32 storage");
        if (p->n_rods > 0 || p->evap_on || p->sink_on)
            return fail(LB_ENOTSUP, "the colour-gradient step takes no rods, reservoir or sink");
        if (!(p->cg_sigma >= 0.0) || !isfinite(p->cg_sigma) || !(p->cg_beta > 0.0 && p->cg_beta <= 1.0) ||
            !(p->cg_grad_eps > 0.0) || !isfinite(p->cg_grad_eps))
            return fail(LB_EINVAL, "colour gradient needs sigma >= 0, 0 < beta <= 1 and grad_eps > 0");
        for (int m = 0; m < LB_NMAT; ++m)
            if (!(p->cg_theta[m] >= 0.0 && p->cg_theta[m] <= M_PI))
                return fail(LB_EINVAL, "contact angle of material %d outside [0, pi]", m);
    }
    if (p->n_fil < 0 || p->fil_beads < 0) return fail(LB_EINVAL, "negative filament count");
    if (p->n_fil > 0) {
        if (p->fil_beads < 1) return fail(LB_EINVAL, "filaments need at least one bead each");
        if (int64_t(p->n_fil) * p->fil_beads > LB_FIL_MAX_BEADS)
            return fail(LB_EINVAL, "%lld beads exceed LB_FIL_MAX_BEADS = %d", (long long)p->n_fil * p->fil_beads,
                        LB_FIL_MAX_BEADS);
        if (p->prec != LB_F64 && p->prec != LB_F32) return fail(LB_ENOTSUP, "filaments run with FP64 or FP32 storage");
        if (p->model != LB_MODEL_SC || p->n_rods > 0)
            return fail(LB_ENOTSUP, "filaments run with the Shan-Chen step and without rods");
        if (p->n_sub < 1) return fail(LB_EINVAL, "n_sub must be >= 1");
        if (!(p->fil_d0 > 0.0) || !(p->fil_R_m > 0.0) || !(p->fil_k_s >= 0.0) || !(p->fil_k_b >= 0.0) ||
            !(p->fil_eps >= 0.0) || !(p->fil_eps_coh >= 0.0) || !(p->fil_gamma >= 0.0) || !isfinite(p->fil_kappa_s) ||
            !(p->fil_mu >= 0.0) || !(p->fil_skin > 0.0) || !(p->fil_eps_s >= 0.0))
            return fail(LB_EINVAL, "bad filament parameters");
        if (p->fil_eps_coh > 0.0 && !(p->fil_r_cut > p->fil_d0)) return fail(LB_EINVAL, "cohesion cut-off must exceed d0");
        if (p->wall_on && (!(p->fil_sigma_s > 0.0) || !(p->fil_r_cut_s > 0.0)))
            return fail(LB_EINVAL, "bad substrate interaction");
    }
    // the integrator keeps 13 doubles per rod in one work-group's shared memory
    if (p->n_rods < 0 || p->n_rods > LB_MAX_RODS)
        return fail(LB_EINVAL, "n_rods = %d outside [0, %d]", p->n_rods, LB_MAX_RODS);
    if (p->n_rods > 0) {
        if (!(p->rod_radius > 0.0) || !(p->rod_length >= 2.0 * p->rod_radius) || !(p->rod_rho > 0.0))
            return fail(LB_EINVAL, "bad rod shape or density");
        if (p->n_sub < 1) return fail(LB_EINVAL, "n_sub must be >= 1");
        if (!(p->rod_d0 > 0.0) || (p->eps_att > 0.0 && !(p->rod_rcut > p->rod_d0)))
            return fail(LB_EINVAL, "bad rod contact distance or cutoff");
        if (p->wall_on && !(p->rod_d0_wall > 0.0)) return fail(LB_EINVAL, "bad rod-wall contact distance");
    }
    return LB_OK;
}

int validate_material(const lb_params *p, const uint8_t *m) {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    auto at = [&](int x, int y, int z) { return m[(int64_t(z) * ny + y) * nx + x]; };
    const int64_t n = nodes(p);
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t v = m[i];
        if (v > MAT_ROD) return fail(LB_EINVAL, "material code %u at node %lld out of range", v, (long long)i);
        if (v == MAT_ROD) return fail(LB_EINVAL, "rod nodes are placed by the rod module, not by lb_init");
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint8_t v = at(x, y, z);
                if (v == MAT_GHOST && !(p->evap_on && z == nz - 1))
                    return fail(LB_EINVAL, "reservoir node off the top plane (%d,%d,%d)", x, y, z);
                if (v != MAT_FLUID) continue;
                if (!p->periodic[0] && (x == 0 || x == nx - 1))
                    return fail(LB_EINVAL, "fluid node on a closed x end plane");
                if (!p->periodic[1] && (y == 0 || y == ny - 1))
                    return fail(LB_EINVAL, "fluid node on a closed y end plane");
                if (!p->periodic[2] && (z == 0 || z == nz - 1))
                    return fail(LB_EINVAL, "fluid node on a closed z end plane");
            }
    if (p->evap_on) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                if (at(x, y, nz - 1) != MAT_GHOST) return fail(LB_EINVAL, "evaporation needs the whole top plane as reservoir");
        if (p->periodic[2]) return fail(LB_EINVAL, "evaporation needs z non-periodic");
    }
    return LB_OK;
}

}  // namespace

struct lb_ctx;
static void apply_tiles(lb_ctx *c, int tile_y, int rows_per_thread, int zchunk);

struct lb_ctx {
    lb_params p;
    void *f[2];
    int cur;
    uint8_t *mat;
    double *ledger;
    unsigned *status;
    double *partials;
    double *result;
    double *psi;
    double *carry;
    double *rods;
    int16_t *rodid;
    int *newid;
    double *rodsum;
    double *rodpart;
    int *shell, *shell_cnt, *nbr_cnt;
    int16_t *nbr;
    char *obs;
    RodArgs *rodargs_dev;      // rod records with f = f[0] and f = f[1]
    void *rho;                 // [2][fs] fluid densities for the rod passes (lattices with rods)
    void *cg;                  // colour-gradient step: colour [fs] and normal [4][fs], or null
    int rho_fresh;             // rho holds the densities of the current state
    double *fil;               // filament bead records, or null
    int *fil_sten, *fil_nbr, *fil_cnt, *fil_claim;
    long long *fil_grid;
    long long *fil_led;        // [2] reservoir ledger change from the filament impulses (2^-50 units)
    int fil_ready;             // lb_fil_set has uploaded the beads
    RodArgs rodargs_host[2];
    double psi_host[32];
    TileCfg tile;
    int ntx, nty, nzc, zchunk;
    int nledger;
    int nslots;    // ledger slot pairs (reservoir tiles, then sink work-groups)
    int32_t *hbuf; // [2][nz][nx*ny] sink column heights per z chunk, or null
    int max_tiles;
    int64_t steps;
    int64_t fs;
    double rref[2];  // storage reference density of the precision form
};

static RodArgs rod_args(lb_ctx *c);
static hipError_t sink_heights(lb_ctx *c, hipStream_t s);

// tile bookkeeping of a context (no device work)
static void apply_tiles(lb_ctx *c, int tile_y, int rows_per_thread, int zchunk) {
    const lb_params *p = &c->p;
    c->tile.tile_y = tile_y;
    c->tile.rows_per_thread = rows_per_thread;
    c->ntx = (p->nx + 63) / 64;
    c->nty = (p->ny + tile_y - 1) / tile_y;
    c->nledger = c->ntx * c->nty;
    int zc = zchunk;
    if (zc <= 0) {
        // about two work-groups per CU while marching at least 8 planes
        const int xy = c->ntx * c->nty;
        int nzc = (512 + xy - 1) / xy;
        nzc = std::max(1, std::min(nzc, (p->nz + 7) / 8));
        zc = (p->nz + nzc - 1) / nzc;
    }
    c->zchunk = std::max(1, std::min(zc, p->nz));
    c->nzc = (p->nz + c->zchunk - 1) / c->zchunk;
    c->tile.zchunk = c->zchunk;
}

static RodArgs rod_args(lb_ctx *c) {
    const lb_params &p = c->p;
    RodArgs a{};
    a.f = c->f[c->cur];
    a.rho = c->rho;
    a.rods = c->rods;
    a.shell_cap = p.n_rods > 0 ? rod_shell_cap(p) : 0;
    a.nblk = p.n_rods > 0 ? rod_nblk(p) : 0;
    a.shell = c->shell;
    a.shell_cnt = c->shell_cnt;
    a.nbr = c->nbr;
    a.nbr_cnt = c->nbr_cnt;
    const size_t np = size_t(std::max(p.n_rods, 0)) * a.nblk * ROD_PART;
    a.part_adh = c->rodpart;
    a.part_upd = c->rodpart + np;
    a.part_link = c->rodpart + 2 * np;
    a.rodid = c->rodid;
    a.newid = c->newid;
    a.mat = c->mat;
    a.status = c->status;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.px = p.periodic[0];
    a.py = p.periodic[1];
    a.pz = p.periodic[2];
    a.fs = c->fs;
    a.n_rods = p.n_rods;
    a.n_sub = p.n_sub;
    a.radius = p.rod_radius;
    a.half = 0.5 * (p.rod_length - 2.0 * p.rod_radius);
    // solid cylinder of length L and radius R
    a.mass = p.rod_rho * M_PI * p.rod_radius * p.rod_radius * p.rod_length;
    a.Ipar = 0.5 * a.mass * p.rod_radius * p.rod_radius;
    a.Iperp = a.mass * (3.0 * p.rod_radius * p.rod_radius + p.rod_length * p.rod_length) / 12.0;
    a.eps_att = p.eps_att;
    a.eps_rep = p.eps_rep;
    a.d0 = p.rod_d0;
    a.r_cut = p.rod_rcut;
    a.eps_wall = p.eps_wall;
    a.d0_wall = p.rod_d0_wall;
    a.wall_z = p.wall_z;
    a.wall_on = p.wall_on;
    a.G = p.G;
    a.psi_rod[0] = p.psi_solid[MAT_ROD][0];
    a.psi_rod[1] = p.psi_solid[MAT_ROD][1];
    a.rho_ref[0] = c->rref[0];
    a.rho_ref[1] = c->rref[1];
    return a;
}

extern "C" {

int64_t lb_pop_stride(const lb_params *p) {
    if (!p) return 0;
    // pad each array to a multiple of 256 elements plus 64 so that the 38
    // concurrent streams do not start on the same HBM channel
    const int64_t n = nodes(p);
    return ((n + 255) / 256) * 256 + 64;
}

size_t lb_pop_bytes(const lb_params *p) {
    if (!p) return 0;
    return size_t(2 * Q) * size_t(lb_pop_stride(p)) * elem_bytes(p->prec);
}

size_t lb_workspace_bytes(const lb_params *p) {
    if (!p) return 0;
    return ws_layout(p).total;
}

const char *lb_last_error(void) { return g_err.c_str(); }

void lb_abi_sizes(size_t out[10]) {
    out[0] = sizeof(lb_params);
    out[1] = sizeof(lb_buffers);
    out[2] = sizeof(lb_obs);
    out[3] = sizeof(lb_droplet);
    out[4] = sizeof(lb_deposit_spec);
    out[5] = sizeof(lb_graph);
    out[6] = sizeof(lb_conv);
    out[7] = sizeof(lb_kirchhoff_spec);
    out[8] = sizeof(lb_kirchhoff_out);
    out[9] = sizeof(lb_unet);
}

int lb_init(const lb_params *p, const lb_buffers *buf, const double *rho_init_host, const uint8_t *material_host,
            const double *rods_host, hipStream_t stream, lb_ctx **out) {
    if (!out) return fail(LB_EINVAL, "null out");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    if (!buf || !buf->f[0] || !buf->f[1] || !buf->workspace) return fail(LB_EINVAL, "null device buffer");
    if (!rho_init_host || !material_host) return fail(LB_EINVAL, "null initial data");
    if ((reinterpret_cast<uintptr_t>(buf->workspace) & 255) != 0) return fail(LB_EINVAL, "workspace not 256-byte aligned");
    rc = validate_material(p, material_host);
    if (rc) return rc;
    if (p->n_rods > 0 && !rods_host) return fail(LB_EINVAL, "n_rods > 0 needs the rod states");
    std::vector<double> rod_stage(size_t(std::max(p->n_rods, 0)) * ROD_STRIDE, 0.0);
    for (int r = 0; r < p->n_rods; ++r) {
        const double *in = rods_host + 13 * r;
        double qn = 0.0;
        for (int q = 0; q < 4; ++q) qn += in[3 + q] * in[3 + q];
        if (!(qn > 0.5 && qn < 2.0)) return fail(LB_EINVAL, "rod %d: quaternion not normalised", r);
        qn = sqrt(qn);
        double *o = rod_stage.data() + size_t(r) * ROD_STRIDE;
        for (int q = 0; q < 3; ++q) o[ROD_X + q] = in[q];
        for (int q = 0; q < 4; ++q) o[ROD_Q + q] = in[3 + q] / qn;
        for (int q = 0; q < 3; ++q) o[ROD_V + q] = in[7 + q];
        for (int q = 0; q < 3; ++q) o[ROD_L + q] = in[10 + q];
    }

    lb_ctx *c = new (std::nothrow) lb_ctx();
    if (!c) return fail(LB_EINVAL, "out of host memory");
    c->p = *p;
    c->f[0] = buf->f[0];
    c->f[1] = buf->f[1];
    c->cur = 0;
    const WsLayout w = ws_layout(p);
    char *ws = static_cast<char *>(buf->workspace);
    c->mat = reinterpret_cast<uint8_t *>(ws + w.mat);
    c->ledger = reinterpret_cast<double *>(ws + w.ledger);
    c->nslots = w.nslots;
    c->hbuf = p->sink_on ? reinterpret_cast<int32_t *>(ws + w.heights) : nullptr;
    c->status = reinterpret_cast<unsigned *>(ws + w.status);
    c->partials = reinterpret_cast<double *>(ws + w.partials);
    c->result = reinterpret_cast<double *>(ws + w.result);
    c->psi = reinterpret_cast<double *>(ws + w.psi);
    c->carry = reinterpret_cast<double *>(ws + w.carry);
    c->rods = reinterpret_cast<double *>(ws + w.rods);
    c->rodid = reinterpret_cast<int16_t *>(ws + w.rodid);
    c->newid = reinterpret_cast<int *>(ws + w.newid);
    c->rodsum = reinterpret_cast<double *>(ws + w.rodsum);
    c->rodpart = reinterpret_cast<double *>(ws + w.rodpart);
    c->shell = reinterpret_cast<int *>(ws + w.shell);
    c->shell_cnt = reinterpret_cast<int *>(ws + w.shell_cnt);
    c->nbr = reinterpret_cast<int16_t *>(ws + w.nbr);
    c->nbr_cnt = reinterpret_cast<int *>(ws + w.nbr_cnt);
    c->obs = ws + w.obs;
    c->rodargs_dev = reinterpret_cast<RodArgs *>(ws + w.rodargs);
    c->rho = (p->n_rods > 0 || fil_beads(p) > 0) ? static_cast<void *>(ws + w.rho) : nullptr;
    c->fil = fil_beads(p) > 0 ? reinterpret_cast<double *>(ws + w.fil) : nullptr;
    c->fil_sten = reinterpret_cast<int *>(ws + w.fil_sten);
    c->fil_nbr = reinterpret_cast<int *>(ws + w.fil_nbr);
    c->fil_cnt = reinterpret_cast<int *>(ws + w.fil_cnt);
    c->fil_grid = reinterpret_cast<long long *>(ws + w.fil_grid);
    c->fil_claim = reinterpret_cast<int *>(ws + w.fil_claim);
    c->fil_led = reinterpret_cast<long long *>(ws + w.fil_led);
    c->fil_ready = 0;
    c->cg = p->model == LB_MODEL_CG ? static_cast<void *>(ws + w.cg) : nullptr;
    c->rho_fresh = 0;
    for (int m = 0; m < 16; ++m)
        for (int k = 0; k < 2; ++k)
            c->psi_host[2 * m + k] = m == MAT_GHOST ? p->rho_top[k] : (m < LB_NMAT ? p->psi_solid[m][k] : 0.0);
    c->fs = lb_pop_stride(p);
    c->max_tiles = w.max_tiles;
    for (int k = 0; k < 2; ++k) c->rref[k] = p->rho_ref[k];
    apply_tiles(c, p->tile_y ? p->tile_y : 8, p->rows_per_thread ? p->rows_per_thread : 1, p->zchunk);
    c->steps = 0;

    const int64_t n = nodes(p);
    const int per[3] = {p->periodic[0], p->periodic[1], p->periodic[2]};
    auto cleanup = [&](int code) {
        delete c;
        return code;
    };
    // staging: densities go through buffer f[1], which the first step overwrites
    if (lb_pop_bytes(p) < size_t(2 * n) * sizeof(double)) return cleanup(fail(LB_EINVAL, "population buffer too small for staging"));
    double *stage = static_cast<double *>(c->f[1]);
    hipError_t e;
    if ((e = hipMemcpyAsync(stage, rho_init_host, size_t(2 * n) * sizeof(double), hipMemcpyHostToDevice, stream)) != hipSuccess)
        return cleanup(hip_fail(e, "upload densities"));
    if ((e = hipMemcpyAsync(c->mat, material_host, size_t(n), hipMemcpyHostToDevice, stream)) != hipSuccess)
        return cleanup(hip_fail(e, "upload material"));
    if ((e = hipMemsetAsync(c->ledger, 0, size_t(w.nslots) * 2 * sizeof(double), stream)) != hipSuccess)
        return cleanup(hip_fail(e, "clear ledger"));
    if ((e = hipMemsetAsync(c->status, 0, 256, stream)) != hipSuccess) return cleanup(hip_fail(e, "clear status"));
    if ((e = hipMemsetAsync(c->carry, 0, 2 * sizeof(double), stream)) != hipSuccess)
        return cleanup(hip_fail(e, "clear ledger carry"));
    if ((e = hipMemcpyAsync(c->psi, c->psi_host, sizeof c->psi_host, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return cleanup(hip_fail(e, "upload psi table"));
    if ((e = launch_flags(c->mat, p->nx, p->ny, p->nz, per, stream)) != hipSuccess) return cleanup(hip_fail(e, "flags"));
    if ((e = launch_init_populations(p->prec, c->f[0], c->fs, stage, c->mat, n, c->rref, stream)) != hipSuccess)
        return cleanup(hip_fail(e, "init populations"));
    if ((e = launch_slot_fill(p->prec, c->f[0], c->fs, c->mat, p->nx, p->ny, p->nz, per, stream)) != hipSuccess)
        return cleanup(hip_fail(e, "slot fill"));
    if (c->cg && (e = hipMemsetAsync(c->cg, 0, 5 * size_t(c->fs) * (p->prec == LB_F64 ? 8 : 4), stream)) != hipSuccess)
        return cleanup(hip_fail(e, "clear colour arrays"));
    if (p->n_rods > 0) {
        if ((e = hipMemcpyAsync(c->rods, rod_stage.data(), rod_stage.size() * sizeof(double), hipMemcpyHostToDevice,
                                stream)) != hipSuccess)
            return cleanup(hip_fail(e, "upload rods"));
        if ((e = hipMemsetAsync(c->rodid, 0xFF, size_t(n) * sizeof(int16_t), stream)) != hipSuccess)
            return cleanup(hip_fail(e, "clear rod ids"));
        if ((e = hipMemsetAsync(c->rodpart, 0, 3 * size_t(p->n_rods) * rod_nblk(*p) * ROD_PART * sizeof(double), stream)) !=
            hipSuccess)
            return cleanup(hip_fail(e, "clear rod partials"));
        for (int q = 0; q < 2; ++q) {
            c->rodargs_host[q] = rod_args(c);
            c->rodargs_host[q].f = c->f[q];
        }
        if ((e = hipMemcpyAsync(c->rodargs_dev, c->rodargs_host, sizeof(c->rodargs_host), hipMemcpyHostToDevice,
                                stream)) != hipSuccess)
            return cleanup(hip_fail(e, "upload rod records"));
        if ((e = launch_rods_place(p->prec, c->rodargs_host[0], RodBatch{c->rodargs_dev, nullptr}, stream)) !=
            hipSuccess)
            return cleanup(hip_fail(e, "place rods"));
    }
    // the second buffer needs the same wall slots only after the first step
    // writes them; clear it so that stale staging bytes never look like state
    if ((e = hipMemsetAsync(c->f[1], 0, lb_pop_bytes(p), stream)) != hipSuccess) return cleanup(hip_fail(e, "clear f[1]"));
    if (p->sink_on && (e = sink_heights(c, stream)) != hipSuccess) return cleanup(hip_fail(e, "sink heights"));
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return cleanup(hip_fail(e, "init sync"));
    if (p->n_rods > 0) {
        unsigned st = 0;
        if ((e = hipMemcpy(&st, c->status, sizeof st, hipMemcpyDeviceToHost)) != hipSuccess)
            return cleanup(hip_fail(e, "read status"));
        if (st & ST_ROD_WALL)
            return cleanup(fail(LB_EINVAL, "a rod overlaps a wall, the reservoir or a closed end plane"));
        if (st & ST_ROD_LIST) return cleanup(fail(LB_EINVAL, "a rod's surface or neighbour list overflowed"));
    }
    *out = c;
    return LB_OK;
}

}  // extern "C"

// step record of a context whose current state is in buffer cur
static StepArgs step_args(const lb_ctx *c, int cur) {
    const lb_params &p = c->p;
    StepArgs a{};
    a.fsrc = c->f[cur];
    a.fdst = c->f[cur ^ 1];
    a.mat = c->mat;
    a.ledger_part = c->ledger;
    a.status = c->status;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.px = p.periodic[0];
    a.py = p.periodic[1];
    a.pz = p.periodic[2];
    a.fs = c->fs;
    a.ntx = c->ntx;
    a.nty = c->nty;
    a.nzc = c->nzc;
    a.zchunk = c->zchunk;
    a.evap = p.evap_on;
    for (int k = 0; k < 2; ++k) {
        a.tau[k] = p.tau[k];
        a.omega[k] = 1.0 / p.tau[k];
        a.rho_top[k] = p.rho_top[k];
        a.rho_ref[k] = c->rref[k];
    }
    a.G = p.G;
    for (int d = 0; d < 3; ++d) a.g[d] = p.body_force[d];
    a.psi_tab = c->psi;
    if (p.sink_on) {
        const size_t slab = size_t(p.nz) * size_t(p.nx) * p.ny;
        a.sink = 1;
        a.sink_J0 = p.sink_J0;
        a.sink_K = p.sink_K;
        a.sink_h0 = p.sink_h0;
        a.h_read = c->hbuf + size_t(cur) * slab;
        a.h_write = c->hbuf + size_t(cur ^ 1) * slab;
        a.sink_ledger = c->ledger + 2 * size_t(c->max_tiles);
    }
    a.rho_out = c->rho;
    if (p.round_stochastic && (p.prec == LB_F16DEV || p.prec == LB_BF16DEV))
        a.sr_key = (uint32_t(c->steps + 1) * 0x9E3779B1u ^ p.sr_seed) | 1u;  // never 0 (0 = nearest)
    return a;
}

static bool is_tau1(const lb_params &p) { return p.tau[0] == 1.0 && p.tau[1] == 1.0; }

// colour-gradient step record of a context whose current state is in buffer cur
static CGArgs cg_args(const lb_ctx *c, int cur) {
    const lb_params &p = c->p;
    CGArgs a{};
    a.fsrc = c->f[cur];
    a.fdst = c->f[cur ^ 1];
    a.mat = c->mat;
    a.status = c->status;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.px = p.periodic[0];
    a.py = p.periodic[1];
    a.pz = p.periodic[2];
    a.fs = c->fs;
    a.nodes = nodes(&p);
    for (int k = 0; k < 2; ++k) {
        a.omega[k] = 1.0 / p.tau[k];
        a.rho_ref[k] = c->rref[k];
    }
    a.sigma = p.cg_sigma;
    a.beta = p.cg_beta;
    a.grad_eps = p.cg_grad_eps;
    for (int d = 0; d < 3; ++d) a.g[d] = p.body_force[d];
    for (int m = 0; m < 16; ++m) a.cos_theta[m] = m < LB_NMAT ? cos(p.cg_theta[m]) : 0.0;
    const size_t eb = p.prec == LB_F64 ? 8 : 4;
    a.colour = c->cg;
    a.normal = static_cast<char *>(c->cg) + size_t(c->fs) * eb;
    return a;
}

// liquid-node counts per column of the current state into the buffer the
// next step reads (chunk slot 0; the other slots cleared)
static hipError_t sink_heights(lb_ctx *c, hipStream_t s) {
    const lb_params &p = c->p;
    const size_t slab = size_t(p.nz) * size_t(p.nx) * p.ny;
    return launch_sink_heights(p.prec, c->f[c->cur], c->fs, c->mat, p.nx, p.ny, p.nz, c->rref,
                               c->hbuf + size_t(c->cur) * slab, s);
}

extern "C" {

int lb_step(lb_ctx *c, int32_t nsteps, hipStream_t stream) {
    if (!c) return fail(LB_EINVAL, "null ctx");
    if (nsteps < 0) return fail(LB_EINVAL, "negative step count");
    const lb_params &p = c->p;
    const bool tau1 = is_tau1(p);
    for (int s = 0; s < nsteps; ++s) {
        hipError_t e = p.model == LB_MODEL_CG ? launch_cg_step(p.prec, cg_args(c, c->cur), stream)
                                              : launch_sc_step(p.prec, tau1, c->tile, step_args(c, c->cur), stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        c->cur ^= 1;
        c->steps++;
    }
    if (nsteps > 0) c->rho_fresh = c->rho != nullptr;
    return LB_OK;
}


int lb_observables(lb_ctx *c, lb_obs *out, hipStream_t stream) {
    if (!c || !out) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    HIP_TRY(launch_observables(p.prec, c->f[c->cur], c->fs, c->mat, nodes(&p), c->rref, c->ledger,
                               p.sink_on ? c->nslots : c->nledger,
                               c->carry, c->partials, OBS_BLOCKS, c->result, stream),
            "observables");
    double r[OBS_FIELDS];
    double rs[5] = {0, 0, 0, 0, 0};
    unsigned st = 0;
    if (p.n_rods > 0) {
        HIP_TRY(launch_rods_sums(rod_args(c), c->rodsum, stream), "rod sums");
        HIP_TRY(hipMemcpyAsync(rs, c->rodsum, sizeof rs, hipMemcpyDeviceToHost, stream), "copy rod sums");
    }
    long long fl[2] = {0, 0};
    if (c->fil && c->fil_ready)
        HIP_TRY(hipMemcpyAsync(fl, c->fil_led, sizeof fl, hipMemcpyDeviceToHost, stream), "copy filament ledger");
    HIP_TRY(hipMemcpyAsync(r, c->result, sizeof r, hipMemcpyDeviceToHost, stream), "copy observables");
    HIP_TRY(hipMemcpyAsync(&st, c->status, sizeof st, hipMemcpyDeviceToHost, stream), "copy status");
    HIP_TRY(hipStreamSynchronize(stream), "observables sync");
    memset(out, 0, sizeof *out);
    out->step = c->steps;
    out->mass[0] = r[0];
    out->mass[1] = r[1];
    out->ledger[0] = r[2] + double(fl[0]) / FIL_FIX;
    out->ledger[1] = r[3] + double(fl[1]) / FIL_FIX;
    out->momentum[0] = r[4];
    out->momentum[1] = r[5];
    out->momentum[2] = r[6];
    out->max_speed = r[7];
    out->kinetic = r[8];
    out->fluid_nodes = int64_t(r[9]);
    out->status = st;
    out->solid[0] = rs[0];
    out->solid[1] = rs[1];
    for (int q = 0; q < 3; ++q) out->rod_momentum[q] = rs[2 + q];
    if (st & ~ST_NOTICES)
        return fail(LB_EUNSTABLE, "device status word 0x%x (1 NaN, 2 rho <= 0, 4 |u| > 0.3, 8 rod motion, 16 rod at a "
                                  "wall, 32 rod list; 64 far refill is a notice)", st);
    return LB_OK;
}

int lb_export(lb_ctx *c, double *rho_dev, double *f_dev, hipStream_t stream) {
    if (!c) return fail(LB_EINVAL, "null ctx");
    const lb_params &p = c->p;
    HIP_TRY(launch_export(p.prec, c->f[c->cur], c->fs, c->mat, nodes(&p), c->rref, rho_dev, f_dev, stream), "export");
    HIP_TRY(hipStreamSynchronize(stream), "export sync");
    return LB_OK;
}

int lb_droplet_shape(lb_ctx *c, double xc, double yc, lb_droplet *out, hipStream_t stream) {
    if (!c || !out) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    const double rx = nearbyint(xc), ry = nearbyint(yc);  // half to even
    if (!(rx >= 0 && rx < p.nx && ry >= 0 && ry < p.ny)) return fail(LB_EINVAL, "centre (%g, %g) off the lattice", xc, yc);
    const ObsLayout l = obs_layout(&p);
    ObsArgs o{};
    o.mat = c->mat;
    o.fs = c->fs;
    o.nx = p.nx;
    o.ny = p.ny;
    o.nz = p.nz;
    o.ix = int(rx);
    o.iy = int(ry);
    o.rho_ref[0] = c->rref[0];
    o.rho_ref[1] = c->rref[1];
    o.col_h = reinterpret_cast<double *>(c->obs + l.col_h);
    o.col_wet = reinterpret_cast<int *>(c->obs + l.col_wet);
    o.line_x = reinterpret_cast<double *>(c->obs + l.line_x);
    o.line_y = reinterpret_cast<double *>(c->obs + l.line_y);
    o.out = reinterpret_cast<double *>(c->obs + l.out);
    HIP_TRY(launch_droplet(p.prec, c->f[c->cur], o, stream), "droplet shape");
    double r[6];
    HIP_TRY(hipMemcpyAsync(r, o.out, sizeof(r), hipMemcpyDeviceToHost, stream), "copy droplet");
    HIP_TRY(hipStreamSynchronize(stream), "droplet sync");
    out->height = r[0];
    out->r_x = r[1];
    out->r_y = r[2];
    out->theta_x = r[3];
    out->theta_y = r[4];
    out->wet_nodes = int64_t(r[5]);
    return LB_OK;
}

int lb_pressure(lb_ctx *c, const int32_t *xyz, int32_t n, double *p_out, hipStream_t stream) {
    if (!c || !xyz || !p_out || n < 0) return fail(LB_EINVAL, "null argument or negative count");
    if (n > PROBE_MAX) return fail(LB_EINVAL, "at most %d probes per call", PROBE_MAX);
    if (n == 0) return LB_OK;
    const lb_params &p = c->p;
    for (int q = 0; q < n; ++q)
        if (xyz[3 * q] < 0 || xyz[3 * q] >= p.nx || xyz[3 * q + 1] < 0 || xyz[3 * q + 1] >= p.ny || xyz[3 * q + 2] < 0 ||
            xyz[3 * q + 2] >= p.nz)
            return fail(LB_EINVAL, "probe %d off the lattice", q);
    const ObsLayout l = obs_layout(&p);
    int *dxyz = reinterpret_cast<int *>(c->obs + l.probe_xyz);
    double *dp = reinterpret_cast<double *>(c->obs + l.probe_p);
    HIP_TRY(hipMemcpyAsync(dxyz, xyz, size_t(3) * n * sizeof(int32_t), hipMemcpyHostToDevice, stream), "copy probes");
    HIP_TRY(launch_pressure(p.prec, c->f[c->cur], c->fs, c->mat, p.nx, p.ny, p.nz, c->rref, p.G, dxyz, n, dp, stream),
            "pressure");
    HIP_TRY(hipMemcpyAsync(p_out, dp, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, stream), "copy pressure");
    HIP_TRY(hipStreamSynchronize(stream), "pressure sync");
    return LB_OK;
}

// deposit arguments of a context for a spec (validated); nb_out: beads per rod
static int deposit_args(lb_ctx *c, const lb_deposit_spec *s, DepArgs &d) {
    const lb_params &p = c->p;
    if (s->n_bins_x < 1 || s->n_bins_x > DEP_MAXBIN || s->n_bins_y < 1 || s->n_bins_y > DEP_MAXBIN)
        return fail(LB_EINVAL, "bins per profile must be in [1, %d]", DEP_MAXBIN);
    if (!(s->bead_spacing > 0) || !(s->r_contact >= 0) || !(s->strip_x >= 0) || !(s->strip_y >= 0))
        return fail(LB_EINVAL, "bad deposit spec");
    const double half = 0.5 * p.rod_length - p.rod_radius;
    const double nbd = floor(2.0 * half / s->bead_spacing + 0.5) + 1.0;
    const int nb = nbd < 2.0 ? 2 : (nbd > DEP_NB ? DEP_NB + 1 : int(nbd));
    if (nb > DEP_NB) return fail(LB_EINVAL, "more than %d beads per rod", DEP_NB);
    const ObsLayout l = obs_layout(&p);
    d = DepArgs{};
    d.rods = c->rods;
    d.n_rods = p.n_rods;
    d.nb = nb;
    d.nbx = s->n_bins_x;
    d.nby = s->n_bins_y;
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.px = p.periodic[0];
    d.py = p.periodic[1];
    d.pz = p.periodic[2];
    d.half = half;
    d.xc = s->xc;
    d.yc = s->yc;
    d.strip_x = s->strip_x;
    d.strip_y = s->strip_y;
    d.r_contact = s->r_contact;
    d.x_src = s->x_src;
    d.x_snk = s->x_snk;
    d.bins = reinterpret_cast<int16_t *>(c->obs + l.bins);
    d.sval = reinterpret_cast<double *>(c->obs + l.sval);
    d.out = reinterpret_cast<double *>(c->obs + l.dep_out);
    d.labels = reinterpret_cast<int32_t *>(c->obs + l.labels);
    d.graph = reinterpret_cast<int32_t *>(c->obs + l.graph);
    return LB_OK;
}

int lb_deposit(lb_ctx *c, const lb_deposit_spec *s, double *g_x, double *s_x, int32_t *n_x, double *g_y, double *s_y,
               int32_t *n_y, int32_t *labels, lb_graph *graph, hipStream_t stream) {
    if (!c || !s || !g_x || !s_x || !n_x || !g_y || !s_y || !n_y || !graph) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    DepArgs d;
    const int rc = deposit_args(c, s, d);
    if (rc != LB_OK) return rc;
    HIP_TRY(launch_deposit(d, stream), "deposit");
    std::vector<double> res(6 * DEP_MAXBIN);
    int32_t gr[4];
    std::vector<int32_t> lab(size_t(std::max(p.n_rods, 0)));
    HIP_TRY(hipMemcpyAsync(res.data(), d.out, res.size() * sizeof(double), hipMemcpyDeviceToHost, stream), "copy deposit");
    HIP_TRY(hipMemcpyAsync(gr, d.graph, sizeof(gr), hipMemcpyDeviceToHost, stream), "copy graph");
    if (!lab.empty())
        HIP_TRY(hipMemcpyAsync(lab.data(), d.labels, lab.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream),
                "copy labels");
    HIP_TRY(hipStreamSynchronize(stream), "deposit sync");
    // Eq. 14 with equal bins: counts over the mean count per bin
    auto finish = [&](const double *r, int nbins, double *g, double *sv, int32_t *ns) {
        double tot = 0.0;
        for (int b = 0; b < nbins; ++b) tot += r[b];
        const double mean = tot / nbins;
        for (int b = 0; b < nbins; ++b) {
            g[b] = mean > 0.0 ? r[b] / mean : 0.0;
            sv[b] = r[DEP_MAXBIN + b];
            ns[b] = int32_t(r[2 * DEP_MAXBIN + b]);
        }
    };
    finish(res.data(), s->n_bins_x, g_x, s_x, n_x);
    finish(res.data() + 3 * DEP_MAXBIN, s->n_bins_y, g_y, s_y, n_y);
    graph->n_rods = gr[0];
    graph->edges = gr[1];
    graph->largest = gr[2];
    graph->spanning = gr[3];
    if (labels)
        for (size_t r = 0; r < lab.size(); ++r) labels[r] = lab[r];
    return LB_OK;
}

int lb_deposit_ensemble(lb_ctx *const *ctxs, int32_t n_runs, const lb_deposit_spec *s, int32_t mirror, double *g_x,
                        double *s_x, int32_t *n_x, double *g_y, double *s_y, int32_t *n_y, hipStream_t stream) {
    if (!ctxs || n_runs < 1 || !s || !g_x || !s_x || !n_x || !g_y || !s_y || !n_y)
        return fail(LB_EINVAL, "null argument or no runs");
    for (int r = 0; r < n_runs; ++r) {
        if (!ctxs[r]) return fail(LB_EINVAL, "null run %d", r);
        const lb_params &a = ctxs[r]->p, &b = ctxs[0]->p;
        if (a.nx != b.nx || a.ny != b.ny || a.periodic[0] != b.periodic[0] || a.periodic[1] != b.periodic[1] ||
            a.rod_length != b.rod_length || a.rod_radius != b.rod_radius)
            return fail(LB_EINVAL, "run %d differs from run 0 in lattice extent, periodicity or rod shape", r);
    }
    const ObsLayout l0 = obs_layout(&ctxs[0]->p);
    double *acc = reinterpret_cast<double *>(ctxs[0]->obs + l0.ens_acc);
    double *out = reinterpret_cast<double *>(ctxs[0]->obs + l0.ens_out);
    HIP_TRY(hipMemsetAsync(acc, 0, 8 * DEP_MAXBIN * sizeof(double), stream), "clear ensemble sums");
    const int nimg = mirror ? 4 : 1;
    for (int r = 0; r < n_runs; ++r) {
        DepArgs d;
        const int rc = deposit_args(ctxs[r], s, d);
        if (rc != LB_OK) return rc;
        for (int m = 0; m < nimg; ++m) {
            d.mirror_x = m & 1;
            d.mirror_y = (m >> 1) & 1;
            HIP_TRY(launch_deposit_accumulate(d, acc, stream), "deposit image");
        }
    }
    HIP_TRY(launch_deposit_finish(acc, s->n_bins_x, s->n_bins_y, n_runs * nimg, out, stream), "deposit ensemble");
    std::vector<double> res(6 * DEP_MAXBIN);
    HIP_TRY(hipMemcpyAsync(res.data(), out, res.size() * sizeof(double), hipMemcpyDeviceToHost, stream),
            "copy ensemble");
    HIP_TRY(hipStreamSynchronize(stream), "ensemble sync");
    for (int b = 0; b < s->n_bins_x; ++b) {
        g_x[b] = res[b];
        s_x[b] = res[DEP_MAXBIN + b];
        n_x[b] = int32_t(res[2 * DEP_MAXBIN + b]);
    }
    for (int b = 0; b < s->n_bins_y; ++b) {
        g_y[b] = res[3 * DEP_MAXBIN + b];
        s_y[b] = res[4 * DEP_MAXBIN + b];
        n_y[b] = int32_t(res[5 * DEP_MAXBIN + b]);
    }
    return LB_OK;
}

int lb_rod_map(lb_ctx *c, int32_t *map_host, hipStream_t stream) {
    if (!c || !map_host) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    const ObsLayout l = obs_layout(&p);
    int32_t *map = reinterpret_cast<int32_t *>(c->obs + l.map);
    HIP_TRY(launch_rod_map(c->mat, p.nx, p.ny, p.nz, map, stream), "rod map");
    HIP_TRY(hipMemcpyAsync(map_host, map, size_t(p.nx) * p.ny * sizeof(int32_t), hipMemcpyDeviceToHost, stream),
            "copy rod map");
    HIP_TRY(hipStreamSynchronize(stream), "rod map sync");
    return LB_OK;
}

static bool canvas_fits(const lb_params &p, int D, int H, int W) {
    return D > 0 && H > 0 && W > 0 && p.nx % 2 == 0 && p.ny % 2 == 0 && p.nz % 2 == 0 && p.nx / 2 <= W &&
           p.ny / 2 <= H && p.nz / 2 <= D;
}

}  // extern "C"

// Restriction and lift read the Shan-Chen force of the state they read or
// write.  Its psi field goes to the context's other population buffer: between
// steps that buffer holds nothing the next step reads before writing it (the
// step rewrites every fluid node and every wall and rod slot), and it holds at
// least 38 x 2 bytes per node, more than the 16 the field takes.
static SurLattice sur_lattice(lb_ctx *c) {
    const lb_params &p = c->p;
    SurLattice L{};
    L.mat = c->mat;
    L.nx = p.nx;
    L.ny = p.ny;
    L.nz = p.nz;
    L.px = p.periodic[0];
    L.py = p.periodic[1];
    L.pz = p.periodic[2];
    L.fs = c->fs;
    for (int k = 0; k < 2; ++k) {
        L.rref[k] = c->rref[k];
        L.tau[k] = p.tau[k];
    }
    L.G = p.G;
    for (int d = 0; d < 3; ++d) L.g[d] = p.body_force[d];
    L.psi_tab = c->psi;
    L.psi = static_cast<double *>(c->f[c->cur ^ 1]);
    return L;
}

extern "C" {

int lb_sur_restrict(lb_ctx *c, int32_t D, int32_t H, int32_t W, float *coarse_f32, void *coarse_bf16,
                    hipStream_t stream) {
    if (!c || (!coarse_f32 && !coarse_bf16)) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    if (!canvas_fits(p, D, H, W)) return fail(LB_EINVAL, "lattice %dx%dx%d does not fit the canvas", p.nx, p.ny, p.nz);
    HIP_TRY(launch_restrict(p.prec, c->f[c->cur], sur_lattice(c), D, H, W, coarse_f32,
                            static_cast<uint16_t *>(coarse_bf16), stream),
            "restrict");
    return LB_OK;
}

int lb_sur_lift(lb_ctx *c, const float *coarse_f32, int32_t D, int32_t H, int32_t W, hipStream_t stream) {
    if (!c || !coarse_f32) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    if (!canvas_fits(p, D, H, W)) return fail(LB_EINVAL, "lattice %dx%dx%d does not fit the canvas", p.nx, p.ny, p.nz);
    c->rho_fresh = 0;
    HIP_TRY(launch_lift(p.prec, coarse_f32, D, H, W, sur_lattice(c), c->f[c->cur], stream), "lift");
    const int per[3] = {p.periodic[0], p.periodic[1], p.periodic[2]};
    HIP_TRY(launch_slot_fill(p.prec, c->f[c->cur], c->fs, c->mat, p.nx, p.ny, p.nz, per, stream), "lift slots");
    // moving bounce-back slots of the rods for the lifted state
    if (p.n_rods > 0)
        HIP_TRY(launch_rods_link(p.prec, c->rodargs_host[c->cur], RodBatch{c->rodargs_dev + c->cur, nullptr}, stream),
                "lift rod links");
    if (p.sink_on) HIP_TRY(sink_heights(c, stream), "sink heights");
    return LB_OK;
}

int lb_sur_jump_rods(lb_ctx *c, const float *coarse_now, const float *coarse_next, int32_t D, int32_t H, int32_t W,
                     double steps, hipStream_t stream) {
    if (!c || !coarse_now || !coarse_next) return fail(LB_EINVAL, "null argument");
    const lb_params &p = c->p;
    if (!canvas_fits(p, D, H, W)) return fail(LB_EINVAL, "lattice %dx%dx%d does not fit the canvas", p.nx, p.ny, p.nz);
    if (!(steps >= 0)) return fail(LB_EINVAL, "negative jump length");
    if (p.n_rods == 0) return LB_OK;
    c->rho_fresh = 0;
    const RodArgs &a = c->rodargs_host[c->cur];
    const RodBatch bt{c->rodargs_dev + c->cur, nullptr, 0};
    HIP_TRY(launch_rods_jump(a, bt, coarse_now, coarse_next, D, H, W, steps, stream), "rod jump");
    HIP_TRY(launch_rods_place(p.prec, a, bt, stream), "re-place rods");
    const int per[3] = {p.periodic[0], p.periodic[1], p.periodic[2]};
    HIP_TRY(launch_flags(c->mat, p.nx, p.ny, p.nz, per, stream), "flags after the jump");
    return LB_OK;
}

int lb_sur_drift_rods(lb_ctx *c, const double *x_prev, double factor, hipStream_t stream) {
    if (!c || !x_prev) return fail(LB_EINVAL, "null argument");
    if (!std::isfinite(factor)) return fail(LB_EINVAL, "non-finite drift factor");
    const lb_params &p = c->p;
    if (p.n_rods == 0) return LB_OK;
    c->rho_fresh = 0;
    const RodArgs &a = c->rodargs_host[c->cur];
    const RodBatch bt{c->rodargs_dev + c->cur, nullptr, 0};
    HIP_TRY(launch_rods_drift(a, bt, x_prev, factor, stream), "rod drift");
    HIP_TRY(launch_rods_place(p.prec, a, bt, stream), "re-place rods");
    const int per[3] = {p.periodic[0], p.periodic[1], p.periodic[2]};
    HIP_TRY(launch_flags(c->mat, p.nx, p.ny, p.nz, per, stream), "flags after the drift");
    return LB_OK;
}

static int conv_check(const lb_conv *a, bool fwd) {
    if (!a || !a->x1 || !a->w) return fail(LB_EINVAL, "null convolution argument");
    if (fwd && !a->wt) return fail(LB_EINVAL, "the forward needs the packed weights wt");
    if (a->c1 <= 0 || a->c1 % 8 || a->c2 < 0 || a->c2 % 8 || a->cout <= 0 || a->cout % 8)
        return fail(LB_EINVAL, "channel counts must be positive multiples of 8 (c2 may be 0)");
    if (a->c2 > 0 && !a->x2) return fail(LB_EINVAL, "null x2 with c2 > 0");
    if (a->D < 1 || a->H < 1 || a->W < 1) return fail(LB_EINVAL, "empty volume");
    if (a->up1 && (a->D % 2 || a->H % 2 || a->W % 2)) return fail(LB_EINVAL, "upsampled input needs even sizes");
    const int64_t P = int64_t(a->D) * a->H * a->W;
    if (P * std::max(a->c1 + a->c2, a->cout) >= (int64_t(1) << 31) || int64_t(27) * (a->c1 + a->c2) * a->cout >= (1 << 30))
        return fail(LB_EINVAL, "tensor too large (element offsets are 32-bit)");
    if (fwd && !a->y && !a->yf) return fail(LB_EINVAL, "no output");
    return LB_OK;
}

static ConvArgs conv_args(const lb_conv *a) {
    ConvArgs c{};
    c.x1 = static_cast<const uint16_t *>(a->x1);
    c.c1 = a->c1;
    c.up1 = a->up1 != 0;
    c.x2 = static_cast<const uint16_t *>(a->x2);
    c.c2 = a->c2;
    c.w = static_cast<const uint16_t *>(a->w);
    c.wt = static_cast<const uint16_t *>(a->wt);
    c.b = a->b;
    c.y = static_cast<uint16_t *>(a->y);
    c.yf = a->yf;
    c.D = a->D;
    c.H = a->H;
    c.W = a->W;
    c.cout = a->cout;
    c.relu = a->relu != 0;
    return c;
}

int lb_conv3d_forward(const lb_conv *a, hipStream_t stream) {
    int rc = conv_check(a, true);
    if (rc) return rc;
    HIP_TRY(launch_conv_fwd(conv_args(a), a->acc, stream), "conv forward");
    return LB_OK;
}

int lb_conv3d_backward_data(const lb_conv *a, const void *g, float *dx, hipStream_t stream) {
    int rc = conv_check(a, false);
    if (rc) return rc;
    if (!g || !dx) return fail(LB_EINVAL, "null gradient");
    HIP_TRY(launch_conv_dgrad(conv_args(a), static_cast<const uint16_t *>(g), dx, stream), "conv backward data");
    return LB_OK;
}

int lb_conv3d_backward_weights(const lb_conv *a, const void *g, float *dw, float *db, hipStream_t stream) {
    int rc = conv_check(a, false);
    if (rc) return rc;
    if (!g || !dw) return fail(LB_EINVAL, "null gradient");
    HIP_TRY(launch_conv_wgrad(conv_args(a), static_cast<const uint16_t *>(g), dw, db, stream), "conv backward weights");
    return LB_OK;
}

int lb_conv_pack_weights(const void *w, int32_t cin, int32_t cout, void *wt, hipStream_t stream) {
    if (!w || !wt || cin <= 0 || cout <= 0 || int64_t(27) * cin * cout >= (1 << 30))
        return fail(LB_EINVAL, "bad weight packing");
    HIP_TRY(launch_pack_weights(static_cast<const uint16_t *>(w), cin, cout, static_cast<uint16_t *>(wt), stream),
            "pack weights");
    return LB_OK;
}

int lb_relu_grad(const float *dy, const void *y, int64_t n, int32_t relu, void *g, hipStream_t stream) {
    if (!dy || !g || n < 0 || (relu && !y)) return fail(LB_EINVAL, "bad ReLU gradient");
    if (n == 0) return LB_OK;
    HIP_TRY(launch_relu_grad(dy, static_cast<const uint16_t *>(y), n, relu != 0, static_cast<uint16_t *>(g), stream),
            "relu grad");
    return LB_OK;
}

int lb_pool2(const void *x, int32_t D, int32_t H, int32_t W, int32_t C, void *y, hipStream_t stream) {
    if (!x || !y || D < 2 || H < 2 || W < 2 || D % 2 || H % 2 || W % 2 || C < 1) return fail(LB_EINVAL, "bad pooling");
    HIP_TRY(launch_pool2(static_cast<const uint16_t *>(x), D, H, W, C, static_cast<uint16_t *>(y), stream), "pool");
    return LB_OK;
}

int lb_pool2_backward(const float *gc, const float *skip, int32_t skip_stride, int32_t skip_off, int32_t D, int32_t H,
                      int32_t W, int32_t C, float *g, hipStream_t stream) {
    if (!gc || !g || D < 2 || H < 2 || W < 2 || D % 2 || H % 2 || W % 2 || C < 1 ||
        (skip && (skip_off < 0 || skip_stride < skip_off + C)))
        return fail(LB_EINVAL, "bad pooling gradient");
    HIP_TRY(launch_pool2_back(gc, skip, skip_stride, skip_off, D, H, W, C, g, stream), "pool backward");
    return LB_OK;
}

int lb_up2_backward(const float *g, int32_t stride, int32_t C, int32_t D, int32_t H, int32_t W, float *gc,
                    hipStream_t stream) {
    if (!g || !gc || C < 1 || stride < C || D < 2 || H < 2 || W < 2 || D % 2 || H % 2 || W % 2)
        return fail(LB_EINVAL, "bad upsampling gradient");
    HIP_TRY(launch_up2_back(g, stride, C, D, H, W, gc, stream), "upsample backward");
    return LB_OK;
}

// ---- whole-network surrogate calls ----------------------------------------
namespace {

struct UnetLayer {
    int c1, c2, cout, up1, lvl;
};

// layer L of the forward order (shapes as lb_sur_forward describes)
UnetLayer unet_layer(const lb_unet *n, int L) {
    const int nl = n->nlev;
    if (L < 2 * nl) {
        const int lvl = L / 2, part = L % 2;
        const int cprev = lvl == 0 ? n->cin : n->ch[lvl - 1];
        return {part == 0 ? cprev : n->ch[lvl], 0, n->ch[lvl], 0, lvl};
    }
    if (L == 4 * nl - 2) return {n->ch[0], 0, n->cout, 0, 0};
    const int k = L - 2 * nl, lvl = nl - 2 - k / 2, part = k % 2;
    const int ccoarse = lvl + 1 == nl - 1 ? n->ch[nl - 1] : n->ch[lvl + 1];
    return part == 0 ? UnetLayer{ccoarse, n->ch[lvl], n->ch[lvl], 1, lvl} : UnetLayer{n->ch[lvl], 0, n->ch[lvl], 0, lvl};
}

int unet_enc(int lvl, int part) { return 2 * lvl + part; }
int unet_dec(const lb_unet *n, int lvl, int part) { return 2 * n->nlev + 2 * (n->nlev - 2 - lvl) + part; }

lb_conv unet_conv(const lb_unet *n, int L, const void *x1, const void *x2, void *y, float *yf, int relu) {
    const UnetLayer l = unet_layer(n, L);
    lb_conv c{};
    c.x1 = x1;
    c.c1 = l.c1;
    c.up1 = l.up1;
    c.x2 = x2;
    c.c2 = l.c2;
    c.w = static_cast<const uint16_t *>(n->pb) + n->off_w[L];
    c.wt = static_cast<const uint16_t *>(n->pt) + n->off_w[L];
    c.b = n->p + n->off_b[L];
    c.y = y;
    c.yf = yf;
    c.acc = l.lvl >= 1 ? n->acc : nullptr;
    c.D = n->D >> l.lvl;
    c.H = n->H >> l.lvl;
    c.W = n->W >> l.lvl;
    c.cout = l.cout;
    c.relu = relu;
    return c;
}

int unet_check(const lb_unet *n, const void *x) {
    if (!n || !x) return fail(LB_EINVAL, "null network or input");
    if (n->nlev < 2 || n->nlev > LB_UNET_MAXLEV) return fail(LB_EINVAL, "nlev must be in [2, %d]", LB_UNET_MAXLEV);
    const int m = 1 << (n->nlev - 1);
    if (n->D < m || n->H < m || n->W < m || n->D % m || n->H % m || n->W % m)
        return fail(LB_EINVAL, "canvas must be divisible by 2^(nlev - 1)");
    if (!n->p || !n->g || !n->pb || !n->pt || !n->out || !n->gm || !n->acc) return fail(LB_EINVAL, "null network buffer");
    for (int L = 0; L < 4 * n->nlev - 2; ++L)
        if (!n->act[L]) return fail(LB_EINVAL, "null activation of layer %d", L);
    for (int l = 0; l < n->nlev; ++l) {
        if (!n->gA[l] || !n->gB[l]) return fail(LB_EINVAL, "null gradient scratch of level %d", l);
        if (l < n->nlev - 1 && (!n->pooled[l] || !n->gcat[l])) return fail(LB_EINVAL, "null level %d buffer", l);
    }
    return LB_OK;
}

}  // namespace

int lb_sur_forward(const lb_unet *n, const void *x, hipStream_t stream) {
    int rc = unet_check(n, x);
    if (rc) return rc;
    const int nl = n->nlev;
    const void *h = x;
    for (int lvl = 0; lvl < nl; ++lvl) {
        for (int part = 0; part < 2; ++part) {
            const int L = unet_enc(lvl, part);
            const lb_conv c = unet_conv(n, L, h, nullptr, n->act[L], nullptr, 1);
            if ((rc = lb_conv3d_forward(&c, stream))) return rc;
            h = n->act[L];
        }
        if (lvl < nl - 1) {
            if ((rc = lb_pool2(h, n->D >> lvl, n->H >> lvl, n->W >> lvl, n->ch[lvl], n->pooled[lvl], stream))) return rc;
            h = n->pooled[lvl];
        }
    }
    for (int lvl = nl - 2; lvl >= 0; --lvl) {
        const int La = unet_dec(n, lvl, 0), Lb = unet_dec(n, lvl, 1);
        lb_conv c = unet_conv(n, La, h, n->act[unet_enc(lvl, 1)], n->act[La], nullptr, 1);
        if ((rc = lb_conv3d_forward(&c, stream))) return rc;
        c = unet_conv(n, Lb, n->act[La], nullptr, n->act[Lb], nullptr, 1);
        if ((rc = lb_conv3d_forward(&c, stream))) return rc;
        h = n->act[Lb];
    }
    const lb_conv c = unet_conv(n, 4 * nl - 2, h, nullptr, nullptr, n->out, 0);
    return lb_conv3d_forward(&c, stream);
}

// gradient of one layer: pre-activation gradient of dy (through the ReLU
// mask of its output y), weight and bias gradients, input gradient into dx
static int unet_layer_grad(const lb_unet *n, int L, const void *x1, const void *x2, const void *y, const float *dy,
                           float *dx, hipStream_t stream) {
    const int relu = L == 4 * n->nlev - 2 ? 0 : 1;
    const lb_conv c = unet_conv(n, L, x1, x2, const_cast<void *>(y), nullptr, relu);
    const int64_t cnt = int64_t(c.D) * c.H * c.W * c.cout;
    int rc;
    if ((rc = lb_relu_grad(dy, y, cnt, relu, n->gm, stream))) return rc;
    if ((rc = lb_conv3d_backward_weights(&c, n->gm, n->g + n->off_w[L], n->g + n->off_b[L], stream))) return rc;
    if (dx) return lb_conv3d_backward_data(&c, n->gm, dx, stream);
    return LB_OK;
}

int lb_sur_backward(const lb_unet *n, const void *x, const float *gout, hipStream_t stream) {
    int rc = unet_check(n, x);
    if (rc) return rc;
    if (!gout) return fail(LB_EINVAL, "null output gradient");
    const int nl = n->nlev;
    float *g = n->gB[0];
    if ((rc = unet_layer_grad(n, 4 * nl - 2, n->act[unet_dec(n, 0, 1)], nullptr, nullptr, gout, g, stream))) return rc;
    // decoder, finest level first: dec{l}b, then dec{l}a whose input is (up(coarse), skip)
    for (int lvl = 0; lvl < nl - 1; ++lvl) {
        float *ga = n->gA[lvl];
        const int La = unet_dec(n, lvl, 0), Lb = unet_dec(n, lvl, 1);
        if ((rc = unet_layer_grad(n, Lb, n->act[La], nullptr, n->act[Lb], g, ga, stream))) return rc;
        const void *coarse = lvl + 1 < nl - 1 ? n->act[unet_dec(n, lvl + 1, 1)] : n->act[unet_enc(nl - 1, 1)];
        const int cup = lvl + 1 < nl - 1 ? n->ch[lvl + 1] : n->ch[nl - 1];
        if ((rc = unet_layer_grad(n, La, coarse, n->act[unet_enc(lvl, 1)], n->act[La], ga, n->gcat[lvl], stream)))
            return rc;
        g = n->gB[lvl + 1];
        if ((rc = lb_up2_backward(n->gcat[lvl], cup + n->ch[lvl], cup, n->D >> lvl, n->H >> lvl, n->W >> lvl, g,
                                  stream)))
            return rc;
    }
    // encoder, coarsest level first
    for (int lvl = nl - 1; lvl >= 0; --lvl) {
        if (lvl < nl - 1) {
            // gradient of enc{lvl}b's output: through the pooling plus the skip
            const int cup = lvl + 1 < nl - 1 ? n->ch[lvl + 1] : n->ch[nl - 1];
            float *gn = n->gA[lvl];
            if ((rc = lb_pool2_backward(g, n->gcat[lvl], cup + n->ch[lvl], cup, n->D >> lvl, n->H >> lvl, n->W >> lvl,
                                        n->ch[lvl], gn, stream)))
                return rc;
            g = gn;
        }
        float *ga = g != n->gB[lvl] ? n->gB[lvl] : n->gA[lvl];
        const int La = unet_enc(lvl, 0), Lb = unet_enc(lvl, 1);
        if ((rc = unet_layer_grad(n, Lb, n->act[La], nullptr, n->act[Lb], g, ga, stream))) return rc;
        const void *xin = lvl == 0 ? x : n->pooled[lvl - 1];
        float *gb = nullptr;
        if (lvl > 0) gb = ga != n->gB[lvl] ? n->gB[lvl] : n->gA[lvl];
        if ((rc = unet_layer_grad(n, La, xin, nullptr, n->act[La], ga, gb, stream))) return rc;
        if (lvl > 0) g = gb;
    }
    return LB_OK;
}

int lb_fill_f32(float *p, int64_t n, float value, hipStream_t stream) {
    if (!p || n < 0) return fail(LB_EINVAL, "bad fill");
    if (n) HIP_TRY(launch_fill_f32(p, n, value, stream), "fill");
    return LB_OK;
}

int lb_to_bf16(const float *x, int64_t n, void *y, hipStream_t stream) {
    if (!x || !y || n < 0) return fail(LB_EINVAL, "bad conversion");
    if (n) HIP_TRY(launch_to_bf16(x, n, static_cast<uint16_t *>(y), stream), "to bf16");
    return LB_OK;
}

static int chan_scale(const float *scale, ChanScale &sc) {
    for (int c = 0; c < 8; ++c) sc.s[c] = 1.0f;
    if (scale)
        for (int c = 0; c < 6; ++c) {
            if (!(scale[c] > 0.0f)) return fail(LB_EINVAL, "channel scale %d must be positive", c);
            sc.s[c] = scale[c];
        }
    return LB_OK;
}

int lb_sur_normalize(const float *x, int64_t P, const float *shift, const float *gain, void *y, hipStream_t stream) {
    if (!x || !y || !shift || !gain || P < 1) return fail(LB_EINVAL, "bad normalisation arguments");
    ChanScale sh, gn;
    for (int c = 0; c < 8; ++c) {
        if (!isfinite(shift[c]) || !isfinite(gain[c])) return fail(LB_EINVAL, "non-finite normalisation");
        sh.s[c] = shift[c];
        gn.s[c] = gain[c];
    }
    HIP_TRY(launch_normalize(x, P, sh, gn, static_cast<uint16_t *>(y), stream), "normalise");
    return LB_OK;
}

int lb_sur_residual(const float *out, const float *xin, int64_t P, const float *scale, float *pred, void *pred_bf16,
                    hipStream_t stream) {
    if (!out || !xin || (!pred && !pred_bf16) || P < 1) return fail(LB_EINVAL, "bad residual arguments");
    ChanScale sc;
    int rc = chan_scale(scale, sc);
    if (rc) return rc;
    HIP_TRY(launch_residual(out, xin, P, sc, pred, static_cast<uint16_t *>(pred_bf16), stream), "residual");
    return LB_OK;
}

size_t lb_sur_loss_scratch_bytes(void) { return SUR_LOSS_SCRATCH * sizeof(double); }

int lb_sur_loss(const float *out, const float *xin, const float *tgt, int64_t P, const float *scale, double lam,
                float *grad, void *scratch, double *result_host, hipStream_t stream) {
    if (!out || !xin || !tgt || !scratch || P < 1) return fail(LB_EINVAL, "bad loss arguments");
    ChanScale sc;
    int rc = chan_scale(scale, sc);
    if (rc) return rc;
    double *part = static_cast<double *>(scratch);
    double *res = part + 256 * 7;
    HIP_TRY(launch_loss(out, xin, tgt, P, sc, lam, part, res, grad, stream), "loss");
    if (result_host) {
        HIP_TRY(hipMemcpyAsync(result_host, res, 4 * sizeof(double), hipMemcpyDeviceToHost, stream), "copy loss");
        HIP_TRY(hipStreamSynchronize(stream), "loss sync");
    }
    return LB_OK;
}

int lb_sur_moments(const float *x, const float *y, int64_t P, void *scratch, double *result_host, hipStream_t stream) {
    if (!x || !y || !scratch || !result_host || P < 1) return fail(LB_EINVAL, "bad moments arguments");
    double *part = static_cast<double *>(scratch);
    double *res = part + 256 * 7;
    HIP_TRY(launch_moments(x, y, P, part, res, stream), "moments");
    HIP_TRY(hipMemcpyAsync(result_host, res, 7 * sizeof(double), hipMemcpyDeviceToHost, stream), "copy moments");
    HIP_TRY(hipStreamSynchronize(stream), "moments sync");
    return LB_OK;
}

int lb_adam(float *p, const float *g, float *m, float *v, void *p_bf16, int64_t n, int32_t step, double lr, double b1,
            double b2, double eps, hipStream_t stream) {
    if (!p || !g || !m || !v || n < 0 || step < 1) return fail(LB_EINVAL, "bad Adam arguments");
    if (n)
        HIP_TRY(launch_adam(p, g, m, v, static_cast<uint16_t *>(p_bf16), n, step, float(lr), float(b1), float(b2),
                            float(eps), stream),
                "adam");
    return LB_OK;
}

int lb_rods_step(lb_ctx *c, hipStream_t stream) {
    if (!c) return fail(LB_EINVAL, "null ctx");
    if (c->p.n_rods == 0) return LB_OK;
    // the rod passes read the fluid step's densities while they describe the
    // current state (the update keeps them so for the nodes it refills), else
    // they sum the populations themselves
    HIP_TRY(launch_rods_step(c->p.prec, RodBatch{c->rodargs_dev + c->cur, nullptr, c->rho_fresh}, 1, c->p.n_rods,
                             rod_nblk(c->p), c->p.n_rods, stream),
            "rods step");
    return LB_OK;
}

int lb_rods_get(lb_ctx *c, double *out_host, hipStream_t stream) {
    if (!c || (!out_host && c->p.n_rods > 0)) return fail(LB_EINVAL, "null argument");
    if (c->p.n_rods == 0) return LB_OK;
    std::vector<double> tmp(size_t(c->p.n_rods) * ROD_STRIDE);
    HIP_TRY(hipMemcpyAsync(tmp.data(), c->rods, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, stream), "copy rods");
    HIP_TRY(hipStreamSynchronize(stream), "rods sync");
    for (int r = 0; r < c->p.n_rods; ++r)
        for (int q = 0; q < 13; ++q) out_host[13 * r + q] = tmp[size_t(r) * ROD_STRIDE + q];
    return LB_OK;
}

static FilArgs fil_args(lb_ctx *c) {
    const lb_params &p = c->p;
    FilArgs a{};
    a.f = c->f[c->cur];
    a.rho = c->rho;
    a.rho_fresh = c->rho_fresh;
    a.mat = c->mat;
    a.psi_tab = c->psi;
    a.bead = c->fil;
    a.sten = c->fil_sten;
    a.nbr = c->fil_nbr;
    a.nbr_cnt = c->fil_cnt;
    a.grid = c->fil_grid;
    a.claim = c->fil_claim;
    a.led = c->fil_led;
    a.evap = p.evap_on;
    a.status = c->status;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.px = p.periodic[0];
    a.py = p.periodic[1];
    a.pz = p.periodic[2];
    a.fs = c->fs;
    a.n = fil_beads(&p);
    a.per_chain = p.fil_beads;
    a.n_sub = p.n_sub;
    a.k_s = p.fil_k_s;
    a.R_m = p.fil_R_m;
    a.eps = p.fil_eps;
    a.d0 = p.fil_d0;
    a.k_b = p.fil_k_b;
    a.eps_coh = p.fil_eps_coh;
    a.r_cut = p.fil_r_cut;
    a.eps_s = p.fil_eps_s;
    a.sigma_s = p.fil_sigma_s;
    a.r_cut_s = p.fil_r_cut_s;
    a.mu = p.fil_mu;
    a.gamma = p.fil_gamma;
    a.kappa_s = p.fil_kappa_s;
    a.mass = M_PI * p.fil_d0 * p.fil_d0 * p.fil_d0 / 6.0;
    a.skin = p.fil_skin;
    a.wall_on = p.wall_on;
    a.wall_z = p.wall_z;
    a.G = p.G;
    for (int d = 0; d < 3; ++d) a.g[d] = p.body_force[d];
    for (int k = 0; k < 2; ++k) {
        a.rho_top[k] = p.rho_top[k];
        a.rho_ref[k] = c->rref[k];
    }
    return a;
}

int lb_fil_set(lb_ctx *c, const double *beads_host, hipStream_t stream) {
    if (!c || !beads_host) return fail(LB_EINVAL, "null argument");
    const int n = fil_beads(&c->p);
    if (n == 0) return fail(LB_EINVAL, "the lattice has no filaments");
    std::vector<double> rec(size_t(n) * FIL_STRIDE, 0.0);
    for (int b = 0; b < n; ++b)
        for (int q = 0; q < 6; ++q) {
            const double v = beads_host[6 * b + q];
            if (!isfinite(v)) return fail(LB_EINVAL, "bead %d: non-finite state", b);
            rec[size_t(b) * FIL_STRIDE + FIL_X + q] = v;  // X then V
        }
    HIP_TRY(hipMemcpyAsync(c->fil, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice, stream), "upload beads");
    HIP_TRY(hipMemsetAsync(c->fil_grid, 0, 3 * size_t(c->fs) * sizeof(long long), stream), "clear momentum grid");
    HIP_TRY(hipMemsetAsync(c->fil_claim, 0x7F, size_t(c->fs) * sizeof(int), stream), "clear owners");  // FIL_NO_OWNER
    HIP_TRY(hipMemsetAsync(c->fil_led, 0, 2 * sizeof(long long), stream), "clear filament ledger");
    HIP_TRY(hipMemsetAsync(c->fil_sten, 0xFF, size_t(n) * 8 * sizeof(int), stream), "clear stencils");
    HIP_TRY(hipStreamSynchronize(stream), "beads sync");
    c->fil_ready = 1;
    return LB_OK;
}

int lb_fil_step(lb_ctx *c, hipStream_t stream) {
    if (!c) return fail(LB_EINVAL, "null ctx");
    if (fil_beads(&c->p) == 0) return LB_OK;
    if (!c->fil_ready) return fail(LB_EINVAL, "lb_fil_set has not been called");
    HIP_TRY(launch_fil_step(c->p.prec, fil_args(c), stream), "filament step");
    return LB_OK;
}

int lb_fil_get(lb_ctx *c, double *out_host, hipStream_t stream) {
    const int n = c ? fil_beads(&c->p) : 0;
    if (!c || (!out_host && n > 0)) return fail(LB_EINVAL, "null argument");
    if (n == 0) return LB_OK;
    std::vector<double> tmp(size_t(n) * FIL_STRIDE);
    HIP_TRY(hipMemcpyAsync(tmp.data(), c->fil, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, stream), "copy beads");
    HIP_TRY(hipStreamSynchronize(stream), "beads sync");
    for (int b = 0; b < n; ++b) {
        const double *r = tmp.data() + size_t(b) * FIL_STRIDE;
        double *o = out_host + 12 * size_t(b);
        for (int q = 0; q < 6; ++q) o[q] = r[FIL_X + q];
        for (int q = 0; q < 3; ++q) o[6 + q] = r[FIL_U + q];
        for (int q = 0; q < 3; ++q) o[9 + q] = r[FIL_IMP + q];
    }
    return LB_OK;
}

int lb_set_tiles(lb_ctx *c, const lb_tile *t, hipStream_t stream) {
    if (!c || !t) return fail(LB_EINVAL, "null argument");
    const bool tau1 = c->p.tau[0] == 1.0 && c->p.tau[1] == 1.0;
    if (!tile_ok(t->tile_y, t->rows_per_thread, tau1))
        return fail(LB_EINVAL, "unsupported tile %d x %d rows per thread", t->tile_y, t->rows_per_thread);
    if (t->zchunk < 0) return fail(LB_EINVAL, "negative zchunk");
    // the ledger slots are indexed by tile: fold them before the layout changes
    HIP_TRY(launch_fold_ledger(c->ledger, c->nslots, c->carry, stream), "fold ledger");
    apply_tiles(c, t->tile_y, t->rows_per_thread, t->zchunk);
    // the sink's column heights are kept per z chunk: count them afresh
    if (c->p.sink_on) HIP_TRY(sink_heights(c, stream), "sink heights");
    return LB_OK;
}

int lb_autotune(lb_ctx *c, int32_t trial_steps, hipStream_t stream, lb_tile *best) {
    if (!c || !best || trial_steps < 1) return fail(LB_EINVAL, "bad autotune arguments");
    if (c->p.model != LB_MODEL_SC) return fail(LB_ENOTSUP, "the colour-gradient step has no tile shape to tune");
    const bool tau1 = c->p.tau[0] == 1.0 && c->p.tau[1] == 1.0;
    const int shapes[4][2] = {{4, 1}, {8, 1}, {8, 2}, {16, 2}};
    const int nz = c->p.nz;
    std::vector<int> chunks;
    for (int zc : {4, 8, 12, 16, 24, 32, 48, 64})
        if (zc <= nz) chunks.push_back(zc);
    if (chunks.empty()) chunks.push_back(nz);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    lb_tile b{0, 0, 0, 1e30};
    int rc = LB_OK;
    for (const auto &sh : shapes) {
        if (!tile_ok(sh[0], sh[1], tau1)) continue;
        for (int zc : chunks) {
            lb_tile t{sh[0], sh[1], zc, 0.0};
            if ((rc = lb_set_tiles(c, &t, stream)) != LB_OK) break;
            if ((rc = lb_step(c, 1, stream)) != LB_OK) break;  // first launch of a shape untimed
            (void)hipEventRecord(e0, stream);
            if ((rc = lb_step(c, trial_steps, stream)) != LB_OK) break;
            (void)hipEventRecord(e1, stream);
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(LB_EHIP, "autotune sync");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double us = 1e3 * ms / trial_steps;
            if (us < b.us_per_step) b = lb_tile{sh[0], sh[1], zc, us};
        }
        if (rc != LB_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LB_OK) return rc;
    rc = lb_set_tiles(c, &b, stream);
    if (rc != LB_OK) return rc;
    *best = b;
    return LB_OK;
}

int lb_current_buffer(const lb_ctx *c) { return c ? c->cur : -1; }

int lb_destroy(lb_ctx *c) {
    delete c;
    return LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches: many lattices advanced by shared launches
// ---------------------------------------------------------------------------
struct lb_batch {
    struct Class {
        TileCfg tile;
        bool tau1;
        int nwork;
        int2 *work;  // device
    };
    std::vector<lb_ctx *> ctx;
    std::vector<int> cur0;  // each lattice's current buffer when the batch was made
    std::vector<Class> classes;
    int prec = 0;
    StepArgs *steps = nullptr;  // device [2][n]: records for batch parity 0 and 1
    RodArgs *rods = nullptr;    // device [2][n]
    int2 *rodmap = nullptr;     // device [total_rods]
    int total_rods = 0, nblk_max = 0, max_rods = 0;
    int par = 0;  // steps taken since creation, mod 2
    hipStream_t cap = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // two steps from parity 0, without / with rods
};

namespace {

struct BatchLayout {
    size_t steps, rods, rodmap, work, total;
    std::vector<size_t> work_off;
};

bool same_tile(const TileCfg &a, const TileCfg &b) { return a.tile_y == b.tile_y && a.rows_per_thread == b.rows_per_thread; }

// class of each lattice (tile shape and tau = 1 select the kernel instance)
std::vector<int> batch_classes(lb_ctx *const *ctxs, int n, std::vector<lb_batch::Class> &cls,
                               std::vector<int> &counts) {
    std::vector<int> of(n);
    for (int i = 0; i < n; ++i) {
        const bool t1 = is_tau1(ctxs[i]->p);
        int k = 0;
        while (k < int(cls.size()) && !(same_tile(cls[k].tile, ctxs[i]->tile) && cls[k].tau1 == t1)) ++k;
        if (k == int(cls.size())) {
            cls.push_back(lb_batch::Class{ctxs[i]->tile, t1, 0, nullptr});
            counts.push_back(0);
        }
        of[i] = k;
        counts[k] += ctxs[i]->ntx * ctxs[i]->nty * ctxs[i]->nzc;
    }
    for (int &c : counts) c = (c + 7) / 8 * 8;  // padded to whole rounds of the eight XCDs
    return of;
}

BatchLayout batch_layout(lb_ctx *const *ctxs, int n) {
    BatchLayout l{};
    std::vector<lb_batch::Class> cls;
    std::vector<int> counts;
    batch_classes(ctxs, n, cls, counts);
    int total_rods = 0;
    for (int i = 0; i < n; ++i) total_rods += ctxs[i]->p.n_rods;
    size_t o = 0;
    l.steps = o;
    o = align256(o + 2 * size_t(n) * sizeof(StepArgs));
    l.rods = o;
    o = align256(o + 2 * size_t(n) * sizeof(RodArgs));
    l.rodmap = o;
    o = align256(o + size_t(total_rods) * sizeof(int2));
    l.work = o;
    for (int c : counts) {
        l.work_off.push_back(o);
        o = align256(o + size_t(c) * sizeof(int2));
    }
    l.total = o;
    return l;
}

int batch_check(lb_ctx *const *ctxs, int n) {
    if (!ctxs || n < 1) return fail(LB_EINVAL, "a batch needs at least one lattice");
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(LB_EINVAL, "null lattice %d", i);
        if (ctxs[i]->p.prec != ctxs[0]->p.prec) return fail(LB_EINVAL, "lattices of a batch share one precision");
        if (ctxs[i]->p.sink_on) return fail(LB_ENOTSUP, "lattice %d uses the evaporation sink, which a batch does not run", i);
        if (ctxs[i]->p.round_stochastic)
            return fail(LB_ENOTSUP, "lattice %d rounds stochastically, which a batch does not run", i);
        if (ctxs[i]->p.model != LB_MODEL_SC)
            return fail(LB_ENOTSUP, "lattice %d runs the colour-gradient step, which a batch does not run", i);
        if (fil_beads(&ctxs[i]->p) > 0)
            return fail(LB_ENOTSUP, "lattice %d carries filaments, which a batch does not run", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(LB_EINVAL, "lattice %d appears twice", i);
    }
    return LB_OK;
}

hipError_t batch_enqueue(lb_batch *b, int par, bool rods, hipStream_t s) {
    const int n = int(b->ctx.size());
    for (const auto &c : b->classes) {
        hipError_t e = launch_sc_step_batch(b->prec, c.tau1, c.tile, b->steps + size_t(par) * n, c.work, c.nwork, s);
        if (e != hipSuccess) return e;
    }
    // the rod update acts on the state the fluid step just wrote: the records
    // of the next parity
    if (rods && b->total_rods > 0)
        return launch_rods_step(b->prec, RodBatch{b->rods + size_t(par ^ 1) * n, b->rodmap, 1}, n, b->total_rods,
                                b->nblk_max, b->max_rods, s);
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t lb_batch_workspace_bytes(lb_ctx *const *ctxs, int32_t n) {
    if (batch_check(ctxs, n) != LB_OK) return 0;
    return batch_layout(ctxs, n).total;
}

int lb_batch_create(lb_ctx *const *ctxs, int32_t n, void *workspace, hipStream_t stream, lb_batch **out) {
    if (!out) return fail(LB_EINVAL, "null out");
    *out = nullptr;
    int rc = batch_check(ctxs, n);
    if (rc) return rc;
    if (!workspace) return fail(LB_EINVAL, "null workspace");
    const BatchLayout l = batch_layout(ctxs, n);
    char *ws = static_cast<char *>(workspace);
    auto *b = new (std::nothrow) lb_batch();
    if (!b) return fail(LB_EINVAL, "out of host memory");
    b->ctx.assign(ctxs, ctxs + n);
    b->prec = ctxs[0]->p.prec;
    std::vector<int> counts;
    const std::vector<int> of = batch_classes(ctxs, n, b->classes, counts);
    b->steps = reinterpret_cast<StepArgs *>(ws + l.steps);
    b->rods = reinterpret_cast<RodArgs *>(ws + l.rods);
    b->rodmap = reinterpret_cast<int2 *>(ws + l.rodmap);
    // per-parity records
    std::vector<StepArgs> sa(2 * size_t(n));
    std::vector<RodArgs> ra(2 * size_t(n));
    std::vector<int2> rmap;
    for (int i = 0; i < n; ++i) {
        lb_ctx *c = ctxs[i];
        b->cur0.push_back(c->cur);
        for (int q = 0; q < 2; ++q) {
            sa[size_t(q) * n + i] = step_args(c, c->cur ^ q);
            ra[size_t(q) * n + i] = rod_args(c);
            ra[size_t(q) * n + i].f = c->f[c->cur ^ q];
        }
        for (int r = 0; r < c->p.n_rods; ++r) rmap.push_back(make_int2(i, r));
        if (c->p.n_rods > 0) {
            b->nblk_max = std::max(b->nblk_max, rod_nblk(c->p));
            b->max_rods = std::max(b->max_rods, c->p.n_rods);
        }
    }
    b->total_rods = int(rmap.size());
    // work lists: each lattice's tiles in its own logical order, the lists of
    // a class concatenated, padded to a multiple of 8 and permuted so that
    // the round-robin dealing of work-groups gives XCD j the j-th eighth
    std::vector<std::vector<int2>> logical(b->classes.size());
    for (int i = 0; i < n; ++i) {
        const int nb = ctxs[i]->ntx * ctxs[i]->nty * ctxs[i]->nzc;
        for (int t = 0; t < nb; ++t) logical[of[i]].push_back(make_int2(i, t));
    }
    hipError_t e = hipSuccess;
    std::vector<std::vector<int2>> hw(b->classes.size());
    for (size_t k = 0; k < b->classes.size(); ++k) {
        const int np = counts[k];
        logical[k].resize(np, make_int2(-1, -1));
        hw[k].resize(np);
        for (int pidx = 0; pidx < np; ++pidx) hw[k][pidx] = logical[k][(pidx & 7) * (np >> 3) + (pidx >> 3)];
        b->classes[k].nwork = np;
        b->classes[k].work = reinterpret_cast<int2 *>(ws + l.work_off[k]);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->classes[k].work, hw[k].data(), np * sizeof(int2), hipMemcpyHostToDevice, stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->steps, sa.data(), sa.size() * sizeof(StepArgs), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->rods, ra.data(), ra.size() * sizeof(RodArgs), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !rmap.empty())
        e = hipMemcpyAsync(b->rodmap, rmap.data(), rmap.size() * sizeof(int2), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the host staging vectors end here
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch set-up");
    }
    *out = b;
    return LB_OK;
}

int lb_batch_step(lb_batch *b, int32_t nsteps, int32_t with_rods, int32_t use_graph, hipStream_t stream) {
    if (!b || nsteps < 0) return fail(LB_EINVAL, "bad batch step arguments");
    const int n = int(b->ctx.size());
    for (int i = 0; i < n; ++i)
        if (b->ctx[i]->cur != (b->cur0[i] ^ b->par))
            return fail(LB_EINVAL, "lattice %d was stepped outside its batch", i);
    const bool rods = with_rods != 0;
    int left = nsteps;
    while (left > 0) {
        if (use_graph && left >= 2 && b->par == 0) {
            hipGraphExec_t &g = b->graph[rods ? 1 : 0];
            if (!g) {
                // capture two steps (parity 0 then 1) once; replays leave every
                // lattice's buffer parity unchanged
                hipGraph_t gr = nullptr;
                HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
                hipError_t e1 = batch_enqueue(b, 0, rods, b->cap);
                hipError_t e2 = e1 == hipSuccess ? batch_enqueue(b, 1, rods, b->cap) : e1;
                hipError_t e3 = hipStreamEndCapture(b->cap, &gr);
                if (e2 != hipSuccess) return hip_fail(e2, "capture batch step");
                if (e3 != hipSuccess) return hip_fail(e3, "end capture");
                hipError_t e4 = hipGraphInstantiate(&g, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e4 != hipSuccess) {
                    g = nullptr;
                    return hip_fail(e4, "instantiate batch graph");
                }
            }
            HIP_TRY(hipGraphLaunch(g, stream), "launch batch graph");
            left -= 2;
        } else {
            HIP_TRY(batch_enqueue(b, b->par, rods, stream), "batch step");
            b->par ^= 1;
            left -= 1;
        }
    }
    for (int i = 0; i < n; ++i) {
        b->ctx[i]->cur ^= (nsteps & 1);
        b->ctx[i]->steps += nsteps;
        // every batch step runs the fluid step, which writes the densities
        if (nsteps > 0) b->ctx[i]->rho_fresh = b->ctx[i]->rho != nullptr;
    }
    return LB_OK;
}

int lb_batch_destroy(lb_batch *b) {
    if (!b) return LB_OK;
    for (auto &g : b->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// resistor network of a deposit
// ---------------------------------------------------------------------------
namespace {

int kirchhoff_check(const double *pos, int32_t n, const lb_kirchhoff_spec *s, double *V, double *I,
                    lb_kirchhoff_out *out) {
    if (!s || !out || n < 0) return fail(LB_EINVAL, "null argument or negative bead count");
    if (n > 0 && (!pos || !V || !I)) return fail(LB_EINVAL, "null bead, potential or current buffer");
    if (n > LB_NET_MAX_BEADS) return fail(LB_EINVAL, "at most %d beads", LB_NET_MAX_BEADS);
    if (!(s->r_c > 0.0) || !std::isfinite(s->r_c) || !std::isfinite(s->x_src) || !std::isfinite(s->x_snk) ||
        !(s->x_src < s->x_snk) || !std::isfinite(s->dV) || !(s->tol > 0.0) || s->max_iter < 0)
        return fail(LB_EINVAL, "bad network spec (r_c > 0, x_src < x_snk, tol > 0, max_iter >= 0, finite values)");
    return LB_OK;
}

// the solve on a workspace of at least net_workspace_bytes(n) bytes
int kirchhoff_run(const double *pos, int32_t n, const lb_kirchhoff_spec *s, double *V, double *I, void *ws,
                  lb_kirchhoff_out *out, hipStream_t stream) {
    memset(out, 0, sizeof *out);
    out->I_ref = s->dV / (s->x_snk - s->x_src);
    if (n == 0) return LB_OK;
    NetArgs a{};
    a.pos = pos;
    a.n = n;
    a.rc2 = s->r_c * s->r_c;
    a.x_src = s->x_src;
    a.x_snk = s->x_snk;
    a.dV = s->dV;
    a.tol = s->tol;
    a.max_iter = s->max_iter;
    a.V = V;
    a.I = I;
    net_carve(a, ws);
    HIP_TRY(launch_net_edges(a, stream), "network edges");
    HIP_TRY(launch_net_solve(a, stream), "network solve");
    double ho[3];
    int hc[4];
    HIP_TRY(hipMemcpyAsync(ho, a.out, sizeof ho, hipMemcpyDeviceToHost, stream), "copy network result");
    HIP_TRY(hipMemcpyAsync(hc, a.cnt, sizeof hc, hipMemcpyDeviceToHost, stream), "copy network counts");
    HIP_TRY(hipStreamSynchronize(stream), "network sync");
    out->I_tot = ho[0];
    out->kappa = out->I_tot / out->I_ref;
    out->rel_residual = ho[1];
    out->iterations = int32_t(ho[2]);
    out->max_degree = hc[0];
    out->n_source = hc[1];
    out->n_sink = hc[2];
    out->edges = hc[3] / 2;
    if (hc[0] > NET_DEG)
        return fail(LB_EINVAL, "a bead has %d neighbours within r_c (at most %d)", hc[0], NET_DEG);
    if (!(ho[1] <= s->tol))
        return fail(LB_EUNSTABLE, "network solve: relative residual %.3e after %d iterations", ho[1], out->iterations);
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lb_kirchhoff_workspace_bytes(int32_t n) { return n <= 0 ? 0 : net_workspace_bytes(size_t(n)); }

int lb_kirchhoff(const double *pos, int32_t n, const lb_kirchhoff_spec *s, double *V, double *I, void *ws,
                 size_t ws_bytes, lb_kirchhoff_out *out, hipStream_t stream) {
    const int rc = kirchhoff_check(pos, n, s, V, I, out);
    if (rc != LB_OK) return rc;
    if (n > 0) {
        if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
            return fail(LB_EINVAL, "network workspace must be a non-null 256-byte aligned device pointer");
        if (ws_bytes < net_workspace_bytes(size_t(n)))
            return fail(LB_EINVAL, "network workspace of %zu bytes, %zu needed for %d beads", ws_bytes,
                        net_workspace_bytes(size_t(n)), int(n));
    }
    return kirchhoff_run(pos, n, s, V, I, ws, out, stream);
}

int lb_kirchhoff_noalloc(const double *pos, int32_t n, const lb_kirchhoff_spec *s, double *V, double *I,
                         lb_kirchhoff_out *out, hipStream_t stream) {
    const int rc = kirchhoff_check(pos, n, s, V, I, out);
    if (rc != LB_OK) return rc;
    if (n > LB_NET_NOALLOC_MAX_BEADS)
        return fail(LB_EINVAL, "lb_kirchhoff_noalloc takes at most %d beads (%d given); use lb_kirchhoff with a "
                               "caller workspace", LB_NET_NOALLOC_MAX_BEADS, int(n));
    void *scratch = nullptr;
    size_t bytes = 0;
    HIP_TRY(net_static_scratch(&scratch, &bytes), "network scratch address");
    if (n > 0 && bytes < net_workspace_bytes(size_t(n)))
        return fail(LB_EINVAL, "network scratch of %zu bytes too small", bytes);
    return kirchhoff_run(pos, n, s, V, I, scratch, out, stream);
}

int lb_rod_beads(lb_ctx *c, double spacing, double *pos, int32_t cap, int32_t *n_out, hipStream_t stream) {
    if (!c || !n_out || cap < 0 || !(spacing > 0.0) || !std::isfinite(spacing))
        return fail(LB_EINVAL, "null argument, negative capacity or bad bead spacing");
    const lb_params &p = c->p;
    const double half = 0.5 * p.rod_length - p.rod_radius;
    const double nbd = floor(2.0 * half / spacing + 0.5) + 1.0;
    const int nb = nbd < 2.0 ? 2 : (nbd > DEP_NB ? DEP_NB + 1 : int(nbd));
    if (nb > DEP_NB) return fail(LB_EINVAL, "more than %d beads per rod", DEP_NB);
    const int64_t n = int64_t(p.n_rods) * nb;
    *n_out = int32_t(n);
    if (n == 0) return LB_OK;
    if (!pos || n > cap) return fail(LB_EINVAL, "bead buffer holds %d beads, %lld needed", int(cap), (long long)n);
    HIP_TRY(launch_rod_beads(c->rods, p.n_rods, nb, half, pos, stream), "rod beads");
    return LB_OK;
}

}  // extern "C"
