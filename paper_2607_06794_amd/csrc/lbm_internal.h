// Internal declarations shared by the HIP translation units of liblbm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// Arguments of the fused step kernel (passed by value as kernel arguments).
struct StepArgs {
    const void *fsrc;
    void *fdst;
    const uint8_t *mat;
    double *ledger_part;  // [nty*ntx][2] running FP64 sums, one slot per xy tile
    unsigned *status;
    int nx, ny, nz;
    int px, py, pz;
    int64_t fs;  // elements between population arrays
    int ntx, nty, nzc, zchunk;
    int evap;
    double tau[2], omega[2];
    double G;
    double g[3];
    const double *psi_tab;  // [16][2] ghost pseudo-densities per material id (device)
    double rho_top[2];
    double rho_ref[2];
    // interfacial evaporation sink (Eq. 8); sink = 0: off
    int sink;
    double sink_J0, sink_K, sink_h0;
    const int32_t *h_read;  // [nz][nx*ny] liquid nodes per column and z chunk of the previous step
    int32_t *h_write;       // the same for this step
    double *sink_ledger;    // [ntx*nty*nzc][2] mass moved A -> B, one running pair per work-group
    void *rho_out;          // [2][fs] fluid densities in compute precision for the rod passes, or null
    uint32_t sr_key;        // 16-bit storage: nonzero = stochastic rounding keyed by this step value
};

// Colour-gradient step (three passes over the lattice; cg_step.hip)
struct CGArgs {
    const void *fsrc;
    void *fdst;
    const uint8_t *mat;
    unsigned *status;
    int nx, ny, nz;
    int px, py, pz;
    int64_t fs;     // elements between population arrays
    int64_t nodes;  // nx * ny * nz
    double omega[2];
    double sigma, beta, grad_eps;
    double g[3];
    double rho_ref[2];
    double cos_theta[16];  // cos of the contact angle per material id
    void *colour;          // [fs] C of every fluid node (compute precision)
    void *normal;          // [4][fs] n_x, n_y, n_z, |grad C| (compute precision)
};
hipError_t launch_cg_step(int prec, const CGArgs &a, hipStream_t s);

// Tile shape of the fused step: TX = 64 columns x tile_y rows, each thread
// owning rows_per_thread rows; the work-group marches zchunk planes.
struct TileCfg {
    int tile_y = 8;
    int rows_per_thread = 2;
    int zchunk = 0;
};

// Rod record: ROD_STRIDE doubles per rod in the workspace
constexpr int ROD_STRIDE = 48;
constexpr int ROD_X = 0, ROD_Q = 3, ROD_V = 7, ROD_L = 10;  // centre, quaternion (w,x,y,z), velocity, ang. momentum
constexpr int ROD_FS = 13, ROD_TS = 16;                      // momentum exchanged by the streamed links
constexpr int ROD_FA = 19, ROD_TA = 22;                      // adhesion reaction
constexpr int ROD_FC = 25, ROD_TC = 28;                      // contact force of the current substep
constexpr int ROD_SOLID = 38;                                // mass exchanged with the fluid [2]
constexpr int ROD_VPRE = 40, ROD_LPRE = 43;                  // momenta the integrator left (before the re-mask transfers)
constexpr int ROD_PART = 8;                                  // doubles per (rod, block) partial-sum slot
constexpr int ROD_NBR = 64;                                  // neighbour-list entries per rod

struct RodArgs {
    void *f;    // current populations (post-collision state)
    void *rho;  // [2][fs] fluid densities of the current state (compute precision)
    double *rods;
    double *part_adh, *part_upd, *part_link;  // [n_rods][nblk][ROD_PART] partial sums
    int *shell;                               // [n_rods][shell_cap] surface-list node indices
    int *shell_cnt;                           // [n_rods]
    int shell_cap, nblk;                      // list capacity; work-groups per rod (shell_cap / 256)
    int16_t *nbr;                             // [n_rods][ROD_NBR] neighbour lists
    int *nbr_cnt;                             // [n_rods]
    int16_t *rodid;  // rod id per node before the move (-1: none)
    int *newid;      // rod id per node after the move
    uint8_t *mat;
    unsigned *status;
    int nx, ny, nz, px, py, pz;
    int64_t fs;
    int n_rods, n_sub;
    double half, radius, mass, Ipar, Iperp;
    double eps_att, eps_rep, d0, r_cut, eps_wall, d0_wall, wall_z;
    int wall_on;
    double G, psi_rod[2], rho_ref[2];
};

// per-lattice rod records on the device; map: global rod -> (lattice, rod),
// null for a single lattice (rod = global index)
struct RodBatch {
    const RodArgs *all;
    const int2 *map;
    int rho_fresh;  // 1: each record's rho holds the densities of its current state
};
// a: host copy of the single lattice's record (sizes, newid), bt its device copy
hipError_t launch_rods_place(int prec, const RodArgs &a, const RodBatch &bt, hipStream_t s);
// one rod update for every lattice of bt: n_lat lattices, total_rods rods,
// nblk_max surface-list work-groups per rod and max_rods rods per lattice at most
hipError_t launch_rods_step(int prec, const RodBatch &bt, int n_lat, int total_rods, int nblk_max, int max_rods,
                            hipStream_t s);
hipError_t launch_rods_sums(const RodArgs &a, double *out, hipStream_t s);
// surrogate jump of one lattice's rods: centres advected by `steps` times the
// mean of the coarse velocities of canvases c0 and c1 ([D][H][W][8]); then all
// rod nodes are returned to fluid (re-place with launch_rods_place)
hipError_t launch_rods_jump(const RodArgs &a, const RodBatch &bt, const float *c0, const float *c1, int D, int H, int W,
                            double steps, hipStream_t s);
// rods continue factor x their displacement since x_prev ([n_rods][3] centres,
// device), relaxed like a jump; re-place with launch_rods_place
hipError_t launch_rods_drift(const RodArgs &a, const RodBatch &bt, const double *x_prev, double factor, hipStream_t s);
hipError_t launch_rods_link(int prec, const RodArgs &a, const RodBatch &bt, hipStream_t s);

// Bead-spring filaments (filaments.hip): bead records FIL_STRIDE doubles
constexpr int FIL_STRIDE = 32;
constexpr int FIL_X = 0, FIL_V = 3;       // position, velocity
constexpr int FIL_U = 6, FIL_GC = 9;      // interpolated fluid velocity and colour gradient of this step
constexpr int FIL_IMP = 12, FIL_X0 = 15;  // impulse given to the fluid this step; position at list time
constexpr int FIL_W = 18;                 // [8] renormalised stencil weights
constexpr int FIL_COUPLED = 26;           // 1 when a stencil node is fluid
constexpr int FIL_XN = 27;                // position slot the substeps alternate with FIL_X
constexpr int FIL_NBR = 48;               // non-bonded partners per bead
constexpr int FIL_MAX = LB_FIL_MAX_BEADS; // beads per lattice
constexpr double FIL_FIX = 1125899906842624.0;  // 2^50: fixed-point unit of the momentum grid and ledger
constexpr int FIL_NO_OWNER = 0x7F7F7F7F;        // empty owner slot (the byte 0x7F repeated)

struct FilArgs {
    void *f;          // current populations (post-collision state)
    const void *rho;  // [2][fs] densities of the current state (compute precision)
    int rho_fresh;    // 1: rho holds them; 0: sum the populations
    const uint8_t *mat;
    const double *psi_tab;  // [16][2] ghost pseudo-densities per material id
    double *bead;           // [n][FIL_STRIDE]
    int *sten;              // [n][8] stencil node indices (-1: none)
    int *nbr, *nbr_cnt;     // [n][FIL_NBR], [n]
    long long *grid;        // [3][fs] momentum per node in units of 2^-50
    int *claim;             // [fs] owner (lowest (bead, stencil) index) of a grid entry waiting to be applied, else FIL_NO_OWNER
    long long *led;         // [2] reservoir ledger change from the impulses, units of 2^-50
    int evap;               // the plane z = nz - 1 is the reservoir
    unsigned *status;
    int nx, ny, nz, px, py, pz;
    int64_t fs;
    int n, per_chain, n_sub;
    double k_s, R_m, eps, d0, k_b, eps_coh, r_cut, eps_s, sigma_s, r_cut_s, mu, gamma, kappa_s, mass, skin;
    int wall_on;
    double wall_z;
    double G, g[3], rho_top[2], rho_ref[2];
};
hipError_t launch_fil_step(int prec, const FilArgs &a, hipStream_t s);

hipError_t launch_sc_step(int prec, bool tau1, const TileCfg &t, const StepArgs &a, hipStream_t s);
// all: device array of per-lattice step records; work: device list of
// (lattice, logical tile) entries, (-1, -1) for padding
hipError_t launch_sc_step_batch(int prec, bool tau1, const TileCfg &t, const StepArgs *all, const int2 *work, int nwork,
                                hipStream_t s);
int tiles_xy(int nx, int ny, int tile_y);

// auxiliary kernels (aux.hip)
hipError_t launch_init_populations(int prec, void *f, int64_t fs, const double *rho, const uint8_t *mat,
                                   int64_t n, const double rho_ref[2], hipStream_t s);
hipError_t launch_flags(uint8_t *mat, int nx, int ny, int nz, const int per[3], hipStream_t s);
hipError_t launch_slot_fill(int prec, void *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz,
                            const int per[3], hipStream_t s);
hipError_t launch_export(int prec, const void *f, int64_t fs, const uint8_t *mat, int64_t n,
                         const double rho_ref[2], double *rho_out, double *f_out, hipStream_t s);
// observables: writes [16] doubles into result (device): mass[2], ledger[2], momentum[3],
// max_speed, kinetic, fluid_nodes
hipError_t launch_observables(int prec, const void *f, int64_t fs, const uint8_t *mat, int64_t n,
                              const double rho_ref[2], const double *ledger_part, int nledger,
                              const double *ledger_carry, double *partials, int nblocks, double *result,
                              hipStream_t s);
hipError_t launch_fold_ledger(double *ledger_part, int nslots, double *carry, hipStream_t s);
// liquid nodes (fluid, rho_A > rho_B) per column of the stored state into h[0][nx*ny];
// chunk slots 1 .. nz-1 of h cleared
hipError_t launch_sink_heights(int prec, const void *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz,
                               const double rho_ref[2], int32_t *h, hipStream_t s);
// droplet shape (column scan) and deposit statistics
struct ObsArgs {
    const uint8_t *mat;
    int64_t fs;
    int nx, ny, nz, ix, iy;
    double rho_ref[2];
    double *col_h;   // [ny][nx] column heights
    int *col_wet;    // [ny][nx] wet nodes per column
    double *line_x;  // [nx] colour on plane z = 1 along row iy
    double *line_y;  // [ny] colour on plane z = 1 along column ix
    double *out;     // h, r_x, r_y, theta_x, theta_y, wet nodes
};
constexpr int DEP_NB = 64;       // beads per rod at most
constexpr int DEP_MAXBIN = 256;  // bins per profile at most
struct DepArgs {
    const double *rods;
    int n_rods, nb, nbx, nby;
    int nx, ny, nz, px, py, pz;
    double half, xc, yc, strip_x, strip_y, r_contact, x_src, x_snk;
    int16_t *bins;   // [n_rods][4][DEP_NB]: bead bin x, bead bin y, segment bin x, segment bin y (-1 outside)
    double *sval;    // [n_rods] 2 e_x^2 - 1
    double *out;     // axial: count, S, segments [3][DEP_MAXBIN]; then transverse, same
    int32_t *labels; // [n_rods] cluster label (smallest rod index of the cluster)
    int32_t *graph;  // n_rods, edges, largest cluster, spanning
    int mirror_x, mirror_y;  // bin the mirror image at (xc, yc): x -> 2 xc - x, y -> 2 yc - y
};
hipError_t launch_droplet(int prec, const void *f, const ObsArgs &o, hipStream_t s);
constexpr int PROBE_MAX = 256;  // pressure probes per call
hipError_t launch_pressure(int prec, const void *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz,
                           const double rref[2], double G, const int *xyz, int n, double *out, hipStream_t s);
hipError_t launch_deposit(const DepArgs &d, hipStream_t s);
// ensemble of deposit profiles: the profiles of d (its mirror flags set) into
// the running sums acc [8][DEP_MAXBIN] (g axial, g transverse, S sums, S
// counts, segment counts); finish turns acc into out [6][DEP_MAXBIN]
// (g_x, S_x, N_x, g_y, S_y, N_y) after `images` accumulations
hipError_t launch_deposit_accumulate(const DepArgs &d, double *acc, hipStream_t s);
hipError_t launch_deposit_finish(const double *acc, int nbx, int nby, int images, double *out, hipStream_t s);

// resistor network of a deposit (network.hip)
constexpr int NET_DEG = 64;  // neighbours stored per bead
struct NetArgs {
    const double *pos;  // [n][3]
    int n;
    double rc2, x_src, x_snk, dV, tol;
    int max_iter;
    int *nbr;      // [n][NET_DEG]
    double *g;     // [n][NET_DEG]
    int *deg;      // [n]
    int *cls;      // [n]: 0 free, 1 source, 2 sink
    double *V, *I; // [n] (caller's)
    double *diag, *r, *z, *p, *q;  // [n] each
    int *cnt;      // max degree, source beads, sink beads, stored directed edges
    double *out;   // I_tot, relative residual, iterations
};
// workspace of one network solve of n beads: neighbour conductances [n][NET_DEG],
// five CG vectors, 8 result doubles, neighbour indices [n][NET_DEG], degree
// and class per bead, 4 counters; rounded up to 256 bytes
constexpr size_t net_workspace_bytes(size_t n) {
    return ((n * NET_DEG * sizeof(double) + 5 * n * sizeof(double) + 8 * sizeof(double) + n * NET_DEG * sizeof(int) +
             2 * n * sizeof(int) + 4 * sizeof(int)) + 255) / 256 * 256;
}
// carve NetArgs' workspace pointers out of ws (256-byte aligned, at least
// net_workspace_bytes(a.n) bytes)
void net_carve(NetArgs &a, void *ws);
hipError_t launch_net_edges(const NetArgs &a, hipStream_t s);
hipError_t launch_net_solve(const NetArgs &a, hipStream_t s);
// device address of the fixed network scratch on the current device (looked
// up once per device) and its size in bytes
hipError_t net_static_scratch(void **ptr, size_t *bytes);
hipError_t launch_rod_beads(const double *rods, int n_rods, int nb, double half, double *pos, hipStream_t s);
hipError_t launch_rod_map(const uint8_t *mat, int nx, int ny, int nz, int32_t *map, hipStream_t s);

// surrogate (surrogate.hip): channels-last BF16 convolutions and helpers
struct ConvArgs {
    const uint16_t *x1;  // channels [0, c1), half resolution when up1
    int c1, up1;
    const uint16_t *x2;  // channels [c1, c1 + c2), full resolution (c2 may be 0)
    int c2;
    const uint16_t *w;   // [27][c1 + c2][cout]
    const uint16_t *wt;  // the same weights packed [cout][27][c1 + c2] (forward)
    const float *b;      // [cout] or null
    uint16_t *y;         // [P][cout] BF16 output (or null)
    float *yf;           // [P][cout] FP32 output (or null)
    int D, H, W, cout, relu;
};
hipError_t launch_conv_fwd(const ConvArgs &a, float *acc, hipStream_t s);
hipError_t launch_conv_dgrad(const ConvArgs &a, const uint16_t *g, float *dx, hipStream_t s);
hipError_t launch_conv_wgrad(const ConvArgs &a, const uint16_t *g, float *dw, float *db, hipStream_t s);
hipError_t launch_pack_weights(const uint16_t *w, int cin, int cout, uint16_t *wt, hipStream_t s);
hipError_t launch_relu_grad(const float *dy, const uint16_t *y, int64_t n, int relu, uint16_t *g, hipStream_t s);
hipError_t launch_pool2(const uint16_t *x, int D, int H, int W, int C, uint16_t *y, hipStream_t s);
hipError_t launch_pool2_back(const float *gc, const float *skip, int skip_stride, int skip_off, int D, int H, int W,
                             int C, float *g, hipStream_t s);
hipError_t launch_up2_back(const float *g, int stride, int C, int D, int H, int W, float *gc, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s);
struct ChanScale {
    float s[8];  // per-channel output scale of the network (channels 0..5)
};
hipError_t launch_normalize(const float *x, int64_t P, const ChanScale &shift, const ChanScale &gain, uint16_t *y,
                            hipStream_t s);
hipError_t launch_residual(const float *out, const float *xin, int64_t P, const ChanScale &sc, float *pred,
                           uint16_t *predb, hipStream_t s);
constexpr int SUR_LOSS_SCRATCH = 256 * 7 + 8;  // doubles
hipError_t launch_loss(const float *out, const float *xin, const float *tgt, int64_t P, const ChanScale &sc, double lam,
                       double *part, double *res, float *grad, hipStream_t s);
hipError_t launch_moments(const float *x, const float *y, int64_t P, double *part, double *res, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s);
// What restriction and lift need of a lattice: geometry, storage and the
// Shan-Chen force parameters; psi is scratch of 2 x nx ny nz doubles
struct SurLattice {
    const uint8_t *mat;
    int nx, ny, nz, px, py, pz;
    int64_t fs;
    double rref[2], tau[2], G, g[3];
    const double *psi_tab;  // [16][2] ghost pseudo-densities per material id (device)
    double *psi;            // [2][nx ny nz] scratch
};
hipError_t launch_restrict(int prec, const void *f, const SurLattice &L, int D, int H, int W, float *outf,
                           uint16_t *outb, hipStream_t s);
hipError_t launch_lift(int prec, const float *coarse, int D, int H, int W, const SurLattice &L, void *f, hipStream_t s);

constexpr int OBS_BLOCKS = 512;
constexpr int OBS_FIELDS = 10;

}  // namespace lbm
