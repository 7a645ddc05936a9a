/*
 * lbm.h -- C ABI of the MI355X drying-droplet lattice Boltzmann library.
 *
 * The library advances a two-component Shan-Chen D3Q19 BGK fluid (lattice
 * Boltzmann equation, Eq. 1; equilibrium, Eq. 2; moments, Eq. 3 of
 * "Evaporation-Driven Nanowire Self-Assembly in an Elongated Droplet",
 * Methods: fluid-filament simulation method) on one AMD Instinct MI355X
 * (gfx950), with halfway bounce-back walls whose ghost pseudo-densities set
 * the wettability (the paper's solid ghost layer for wetting, Methods), a
 * fixed-density reservoir plane on top through which component A evaporates,
 * and rigid capsule rods standing in for the paper's nanowire filaments.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Lattice index: node (x, y, z) has flat index n = (z*ny + y)*nx + x.
 *  - Populations are stored structure-of-arrays, one array per (component k,
 *    direction i), array a = k*19 + i starting at element a*pop_stride, where
 *    pop_stride = lb_pop_stride(params) >= nx*ny*nz.  Element type follows
 *    params.prec (FP64, FP32, IEEE half or bfloat16); every form stores the
 *    deviation f - w_i*rho_ref[k] from the lattice weights (rho_ref = 0
 *    stores f itself).  The stored state at time t is the post-collision
 *    population f*(t); at t = 0 it is w_i*rho_k.
 *  - D3Q19 direction order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 =
 *    (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),
 *    (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *  - Material codes (uint8): 0 fluid, 1 reservoir plane (must be the whole
 *    plane z = nz-1 when evaporation is on), 2..7 static wall materials,
 *    8 rod.  A non-periodic direction must be closed by non-fluid end planes.
 *  - Ownership: every device buffer is allocated and freed by the caller;
 *    the library allocates only its small host-side context.  Buffers must
 *    outlive the context.  The library never calls hipMalloc/hipFree.
 *  - Streams: every call enqueues on the given stream and returns without
 *    synchronising, except lb_init, lb_observables and lb_export which
 *    synchronise that stream before returning.  One context per stream; a
 *    context is not thread-safe.
 *  - Errors: 0 = LB_OK; negative codes below.  No exception crosses the ABI.
 *    lb_last_error() returns a thread-local message for the last failure.
 *    Faults detected inside kernels (NaN, non-positive total density,
 *    |u| > 0.3, rod limits) set a device status word that lb_observables
 *    reports as LB_EUNSTABLE (notice bits alone do not).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LB_OK = 0,
    LB_EINVAL = -1,    /* bad argument: null pointer, size, tau <= 1/2, boundary */
    LB_ENOTSUP = -2,   /* precision or feature combination not supported */
    LB_EHIP = -3,      /* a HIP runtime call failed; see lb_last_error() */
    LB_EUNSTABLE = -4, /* device status word set: NaN, rho <= 0 or |u| > 0.3 */
    LB_EPLACE = 1      /* warning: fewer rods placed than requested */
};

typedef enum { LB_F64 = 0, LB_F32 = 1, LB_F16DEV = 2, LB_BF16DEV = 3 } lb_prec;

#define LB_NMAT 9
#define LB_MAX_RODS 512 /* rods per lattice */
#define LB_FIL_MAX_BEADS 4096 /* filament beads per lattice */

/* All parameters of one lattice (plain data; mirrored by a Python dataclass). */
typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];          /* x, y, z: 1 periodic, 0 closed by non-fluid planes */
    int32_t prec;                 /* lb_prec */
    double tau[2];                /* BGK relaxation time per component, > 1/2 (Eq. 1) */
    double G;                     /* Shan-Chen cross-coupling strength */
    double body_force[3];         /* acceleration g; force rho_k*g */
    double psi_solid[LB_NMAT][2]; /* ghost pseudo-density seen at solid material m */
    int32_t evap_on;              /* 1: plane z = nz-1 is the fixed-density reservoir */
    double rho_top[2];            /* reservoir densities */
    double rho_ref[2];            /* storage reference: arrays hold f_i - w_i*rho_ref[k] (0: f_i) */
    /* rigid rods (capsules): count, shape and interactions */
    int32_t n_rods;               /* rods given to lb_init (0: none, at most LB_MAX_RODS) */
    int32_t n_sub;                /* rigid-body substeps per lattice step (5) */
    double rod_length;            /* tip-to-tip length L */
    double rod_radius;            /* capsule radius R */
    double rod_rho;               /* rod density (mass = rho pi R^2 L) */
    double eps_att;               /* rod-rod cohesion well depth (Eq. 12 form) */
    double eps_rep;               /* rod-rod excluded-volume strength (Eq. 10 form) */
    double rod_d0;                /* contact distance of the segment-segment potentials */
    double rod_rcut;              /* cohesion cutoff (energy shifted to 0 there) */
    double eps_wall;              /* rod-wall excluded volume strength */
    double rod_d0_wall;           /* rod-wall contact distance */
    int32_t wall_on;              /* 1: wall plane at z = wall_z repels rods */
    double wall_z;
    /* tiling of the fused step (0 = library default); see lb_autotune */
    int32_t tile_y;               /* 4, 8 or 16 rows per tile */
    int32_t rows_per_thread;      /* 1 or 2 */
    int32_t zchunk;               /* planes marched by one work-group; 0 = auto */
    /* the paper's evaporation law (Methods, evaporation paragraph; Eq. 8): an
     * interfacial sink with flux J = J0 / (K + h / h0), used instead of (or
     * besides) the reservoir plane.  After each collision, at every
     * interface node -- a fluid node with rho_A > rho_B whose upper
     * neighbour (z + 1) is a fluid node with rho_A < rho_B -- the amount
     * min(J, f*_0^A), at least 0, moves from the rest population of A to
     * that of B and is booked in the ledgers (ledger[0] += moved,
     * ledger[1] -= moved).  h is the number of fluid nodes with
     * rho_A > rho_B in the node's column in the state the step starts from.
     * FP32 storage, or FP64 with tau = 1 (LB_ENOTSUP otherwise); a batch does
 * not take such lattices (LB_ENOTSUP). */
    int32_t sink_on;              /* 1: interfacial sink */
    double sink_J0;               /* flux scale J0 >= 0 */
    double sink_K;                /* kinetic resistance K >= 0 (0.01 in the paper) */
    double sink_h0;               /* initial droplet height h0 > 0 (nodes) */
    /* fluid model: LB_MODEL_SC, the Shan-Chen pseudopotential step (fields
     * above), or LB_MODEL_CG, the paper's colour-gradient step (Methods,
     * fluid-filament paragraphs; Eqs. 1-3): per component BGK (tau[k])
     * towards the equilibrium of the common velocity u = (sum_k j_k + F/2) /
     * rho with Guo's forcing, the capillary force F = (cg_sigma / 2) kappa
     * |grad C| n of the colour field C = (rho_1 - rho_2) / rho (n = grad C /
     * |grad C| where |grad C| > cg_grad_eps, kappa = -div n, both with the
     * isotropic D3Q19 stencil) plus rho * body_force, shared by the
     * components in proportion to their densities, then recolouring
     * f^{1,2}_i = (rho_{1,2} / rho) f*_i +- cg_beta (rho_1 rho_2 / rho) w_i
     * c_i.n / |c_i|.  Wetting: a wall node next to the fluid carries the
     * w-weighted mean colour of its fluid neighbours, and a fluid node next
     * to walls turns its normal to -cos(theta) n_w + sin(theta) t (n_w the
     * wall normal from its solid neighbours, t the unit tangential part of
     * n, theta the w-weighted mean of cg_theta over those neighbours).
     * FP64 or FP32 storage, no rods, reservoir or sink (LB_ENOTSUP). */
    int32_t model;
    double cg_sigma;              /* interfacial tension (lattice units) */
    double cg_beta;               /* recolouring segregation parameter (0, 1] */
    double cg_grad_eps;           /* |grad C| below which the normal is zero */
    double cg_theta[LB_NMAT];     /* contact angle of wall material m (radians, through component 1) */
    /* 16-bit storage forms: 0 round to nearest even, 1 stochastic rounding
     * (the value goes to the upper of its two representable neighbours with
     * probability equal to its distance from the lower one over their
     * spacing; random bits from a xorshift32 stream per node and step,
     * seeded by a hash of node, step and sr_seed and advanced per population
     * array, so they depend on node, array and step only), which keeps the
     * stored errors unbiased.  Only
     * the fused Shan-Chen step rounds stochastically (lb_init, the rod passes
     * and the surrogate's lift round to nearest); a batch does not take such
     * lattices (LB_ENOTSUP). */
    int32_t round_stochastic;
    uint32_t sr_seed;
    /* bead-spring filaments (Methods, filament paragraphs; Eqs. 9-12):
     * n_fil chains of fil_beads beads each (at most LB_FIL_MAX_BEADS beads in
     * all), bead mass pi fil_d0^3 / 6.  Forces on bead a from bead b at
     * distance d along r = x_a - x_b (minimum image), each -dU/dd r / d:
     *   every pair with d <= fil_d0: excluded volume (Eq. 10)
     *     U = fil_eps [(d0/d)^12 - 2 (d0/d)^6] + fil_eps;
     *   neighbours in a chain: FENE (Eq. 9)
     *     U = -1/2 fil_k_s fil_R_m^2 ln(1 - d^2 / fil_R_m^2);
     *   second neighbours in a chain: bending (Eq. 11) U = 1/2 fil_k_b (d - 2 d0)^2;
     *   beads of different chains with d0 < d < fil_r_cut: cohesion
     *     (Eq. 12) U = fil_eps_coh [(d0/d)^12 - 2 (d0/d)^6] (force only);
     *   the wall plane z = wall_z (when wall_on), h = z - wall_z, 0 < h <
     *     fil_r_cut_s: adhesion U = fil_eps_s [(s/h)^12 - 2 (s/h)^6],
     *     s = fil_sigma_s, and friction -v_t min(fil_mu N / |v_t|, m / dt)
     *     on the tangential velocity v_t with the normal load N = max(0,
     *     -(every other z-force + the attractive part of the adhesion));
     *   drag -fil_gamma (V - u) and solvation fil_kappa_s grad C, u and
     *     grad C interpolated (trilinear, weights renormalised over fluid
     *     nodes) from the physical velocity (sum_k j*_k - F/2) / rho and the
     *     lattice gradient 3 sum_i w_i C(x + c_i) c_i of the colour
     *     C = (rho_A - rho_B) / rho of the state after the fluid step, held
     *     over the substeps.
     * n_sub substeps (forces, then V, then X).  The fluid receives the drag's
     * and the solvation's reactions, spread with the same weights, by the
     * exact-difference rule.  Non-bonded partners come from a list built at
     * the start of each update over the range max(d0, r_cut) + fil_skin;
     * a bead moving more than fil_skin / 2 in one update raises status bit 8,
     * a list longer than 48 bit 32.  FP64 or FP32 storage, Shan-Chen model,
     * no rods in the same lattice (LB_ENOTSUP); a batch does not take such
     * lattices. */
    int32_t n_fil;                /* filaments (0: none) */
    int32_t fil_beads;            /* beads per filament */
    double fil_k_s, fil_R_m;      /* FENE spring constant and maximum extension (0.3, 2.4) */
    double fil_eps, fil_d0;       /* excluded volume strength and bead diameter (0.03, 2) */
    double fil_k_b;               /* bending stiffness (8) */
    double fil_eps_coh, fil_r_cut;/* cohesion well depth and cut-off */
    double fil_eps_s, fil_sigma_s, fil_r_cut_s; /* substrate adhesion (0.006), its minimum and cut-off */
    double fil_mu;                /* friction coefficient */
    double fil_gamma, fil_kappa_s;/* drag coefficient, solvation strength */
    double fil_skin;              /* partner-list skin */
} lb_params;

enum { LB_MODEL_SC = 0, LB_MODEL_CG = 1 };

/* Caller-owned device buffers. */
typedef struct {
    void *f[2];        /* two population buffers, lb_pop_bytes() each */
    void *workspace;   /* lb_workspace_bytes() bytes, 256-byte aligned */
} lb_buffers;

/* Host-side results of lb_observables (FP64 reductions over fluid nodes). */
typedef struct {
    int64_t step;          /* steps taken since lb_init */
    double mass[2];        /* sum over fluid nodes of rho_k */
    double ledger[2];      /* mass of component k lost to the reservoir so far */
    double momentum[3];    /* sum over fluid nodes and components of post-collision j */
    double max_speed;      /* max |sum_k j_k / sum_k rho_k| */
    double kinetic;        /* sum of |j|^2 / (2 rho) */
    int64_t fluid_nodes;
    uint32_t status;       /* device status bits (1 NaN, 2 rho <= 0, 4 |u| > 0.3,
                              8 a rod point moved >= 0.9 in one step, 16 a rod
                              reached a wall, the reservoir or a closed end,
                              32 a rod's surface or neighbour list overflowed;
                              notice, not a fault: 64 a node a rod uncovered
                              had no fluid neighbour and took the mean density
                              of a farther ring x + s c_i, 2 <= s <= ceil(2R)+2) */
    double solid[2];       /* mass of component k moved from the fluid into rods */
    double rod_momentum[3];/* sum over rods of M V */
} lb_obs;

typedef struct lb_ctx lb_ctx;

/* Elements between consecutive population arrays (>= nx*ny*nz). */
int64_t lb_pop_stride(const lb_params *p);
/* Bytes of one population buffer: 38 * pop_stride * element size. */
size_t lb_pop_bytes(const lb_params *p);
/* Bytes of the workspace (material map copy, ledger partials, reductions). */
size_t lb_workspace_bytes(const lb_params *p);

/*
 * Create a context and write the t = 0 state f* = w_i rho_k into buffers.f[0].
 *   rho_init_host : host, FP64 [2][nz][ny][nx] initial densities (values on
 *                   non-fluid nodes are ignored).
 *   material_host : host, uint8 [nz][ny][nx] material codes (copied).
 *   rods_host     : host, FP64 [n_rods][13] = centre X (x, y, z), unit
 *                   quaternion q (w, x, y, z) of the rotation taking e_z to the
 *                   axis, velocity V, angular momentum L; nullable when
 *                   n_rods = 0.  Rod nodes are cut out of the fluid.
 * Validates the parameters and the boundary layout (LB_EINVAL), uses
 * buffers.f[1] as upload staging, and synchronises the stream.
 */
int lb_init(const lb_params *p, const lb_buffers *buf, const double *rho_init_host,
            const uint8_t *material_host, const double *rods_host, hipStream_t stream, lb_ctx **out);

/* One rod update after lb_step(1): reaction of the adhesion force, n_sub
 * rigid-body substeps with the momentum exchanged at the links, rod-rod and
 * rod-wall forces, re-mask with cover/uncover, and the moving bounce-back of
 * the next step.  A no-op without rods.  Asynchronous. */
int lb_rods_step(lb_ctx *ctx, hipStream_t stream);

/* Copy the rod states to out_host [n_rods][13] (layout as in lb_init).
 * Synchronises. */
int lb_rods_get(lb_ctx *ctx, double *out_host, hipStream_t stream);

/* Filaments (see lb_params): beads_host [n_fil * fil_beads][6] holds each
 * bead's position (x, y, z) and velocity, bead b of filament f at row
 * f * fil_beads + b.  Uploads them and clears the momentum grid; call once
 * after lb_init (LB_EINVAL without filaments).  Synchronises. */
int lb_fil_set(lb_ctx *ctx, const double *beads_host, hipStream_t stream);

/* One filament update after lb_step(1): interpolate the fluid velocity and
 * colour gradient at the beads, n_sub substeps, hand the reactions back to
 * the stored populations.  A no-op without filaments.  Asynchronous. */
int lb_fil_step(lb_ctx *ctx, hipStream_t stream);

/* Copy per bead [n_beads][12]: position, velocity, the interpolated fluid
 * velocity of the last update and the impulse the fluid received from the
 * bead in it.  Synchronises. */
int lb_fil_get(lb_ctx *ctx, double *out_host, hipStream_t stream);

/* Advance the fluid nsteps >= 0 time steps (pull stream, boundaries, moments,
 * pseudopotential force, velocity shift, BGK collision, store; reservoir
 * ledger).  Asynchronous. */
int lb_step(lb_ctx *ctx, int32_t nsteps, hipStream_t stream);

/* FP64 reductions of the current state into *out (host).  Synchronises.
 * Returns LB_EUNSTABLE if the device status word is set. */
int lb_observables(lb_ctx *ctx, lb_obs *out, hipStream_t stream);

/*
 * Decode the current state to FP64 device arrays (caller-owned):
 *   rho_dev : [2][N] densities (0 on non-fluid nodes), nullable
 *   f_dev   : [2][19][N] post-collision populations (0 on non-fluid), nullable
 * Synchronises.
 */
int lb_export(lb_ctx *ctx, double *rho_dev, double *f_dev, hipStream_t stream);

/*
 * Droplet shape of the current state (Results, drying dynamics: height,
 * footprint radii and contact angles along x and y; the extraction is this
 * library's reading, the paper gives none).  Colour C = (rho_A - rho_B) /
 * (rho_A + rho_B) on fluid nodes, liquid C > 0:
 *   height    : largest column height above the wall surface z = 1/2 (topmost
 *               wet node of the column plus the interpolated C = 0 crossing)
 *   r_x, r_y  : half-lengths of the run of C > 0 on plane z = 1 along the row
 *               y = yc and the column x = xc through the centre node (xc, yc
 *               rounded half to even), ends interpolated at C = 0
 *   theta_x/y : spherical-cap contact angles 2 atan(height / r) [rad]
 *   wet_nodes : fluid nodes with C > 0
 * The centre node must lie in the lattice (LB_EINVAL otherwise).  Synchronises.
 */
typedef struct {
    double height, r_x, r_y, theta_x, theta_y;
    int64_t wet_nodes;
} lb_droplet;
int lb_droplet_shape(lb_ctx *ctx, double xc, double yc, lb_droplet *out, hipStream_t stream);

/*
 * Pressure at probe nodes (Shan-Chen equation of state of the current state,
 * the quantity of the Laplace check): p = c_s^2 (rho_A + rho_B) + G c_s^2
 * psi_A psi_B with psi_k = rho_k, c_s^2 = 1/3.  xyz: host, n x (x, y, z) node
 * coordinates, 0 <= n <= 256; p_out: host, n doubles, NaN at probes that are
 * not fluid nodes.  LB_EINVAL for probes off the lattice.  Synchronises.
 */
int lb_pressure(lb_ctx *ctx, const int32_t *xyz, int32_t n, double *p_out, hipStream_t stream);

/*
 * Deposit statistics of the rods (Methods, structural characterisation,
 * Eqs. 13 and 14).  Each rod is represented by nb = max(2, floor(2 h /
 * bead_spacing + 1/2) + 1) beads evenly spaced along its axis segment
 * (half-length h = L/2 - R; nb <= 64) and the nb - 1 segments between them.
 * Axial profiles bin x into n_bins_x equal bins over [0, nx) for beads and
 * segment midpoints with |y - yc| <= strip_y / 2; transverse profiles bin y
 * into n_bins_y bins over [0, ny) with |x - xc| <= strip_x / 2 (minimum image
 * in periodic directions; 1 <= bins <= 256).  Outputs (host, caller-owned):
 *   g_x[n_bins_x], g_y[n_bins_y] : Eq. 14, bead count over the mean count per
 *                                  bin (all 0 if no bead is binned)
 *   s_x[n_bins_x], s_y[n_bins_y] : Eq. 13, mean of 2 cos^2(zeta_x) - 1 over
 *                                  the segments of the bin (0 if none)
 *   n_x, n_y                     : segments per bin
 *   labels[n_rods] (nullable)    : contact-graph cluster of each rod (its
 *                                  smallest rod index)
 *   graph                        : rods, edges (segment distance < r_contact),
 *                                  largest cluster size, spanning = 1 if one
 *                                  cluster reaches x < x_src and x > x_snk
 * Synchronises.
 */
typedef struct {
    int32_t n_bins_x, n_bins_y;
    double xc, yc, strip_x, strip_y;
    double bead_spacing, r_contact, x_src, x_snk;
} lb_deposit_spec;
typedef struct {
    int32_t n_rods, edges, largest, spanning;
} lb_graph;
int lb_deposit(lb_ctx *ctx, const lb_deposit_spec *spec, double *g_x, double *s_x, int32_t *n_x, double *g_y,
               double *s_y, int32_t *n_y, int32_t *labels, lb_graph *graph, hipStream_t stream);

/*
 * The same profiles averaged over independent runs and, when mirror != 0,
 * over each run's mirror images at the droplet centre (x -> 2 xc - x, y ->
 * 2 yc - y, both): the angle brackets of Eqs. 13 and 14 (Results, nematic
 * order and density profile: profiles averaged over independent runs and
 * their mirror images).  g^b is the mean over all images of each image's
 * normalised bead profile; S_x^b the mean over the images with segments in
 * bin b of their bin means (0 where none has); n_x, n_y the segments per
 * bin summed over the images.  ctxs[0..n_runs) share the lattice extent,
 * periodicity and rod shape (LB_EINVAL otherwise); the sums run on the
 * device in ctxs[0]'s workspace, image after image in run order.  Outputs
 * are host arrays as for lb_deposit.  Synchronises.
 */
int lb_deposit_ensemble(lb_ctx *const *ctxs, int32_t n_runs, const lb_deposit_spec *spec, int32_t mirror,
                        double *g_x, double *s_x, int32_t *n_x, double *g_y, double *s_y, int32_t *n_y,
                        hipStream_t stream);

/* z-projected rod occupancy: rod nodes per (y, x) column into map_host
 * [ny][nx] (host, caller-owned).  Synchronises. */
int lb_rod_map(lb_ctx *ctx, int32_t *map_host, hipStream_t stream);

/*
 * Resistor network of a deposit (Methods, electrical characterisation,
 * Eqs. 15-18).  Nodes are beads; beads i != j with 0 < r_ij^2 < r_c^2
 * (r_ij^2 = (dx^2 + dy^2) + dz^2 in FP64, plain Euclidean: no periodic
 * images) are joined with conductance G_ij = 1 / r_ij.  Beads with
 * x < x_src form the source electrode (potential dV), beads with x > x_snk
 * the sink (potential 0); the other potentials satisfy Kirchhoff's current
 * law, sum_j G_ij (V_i - V_j) = 0, solved by Jacobi-preconditioned conjugate
 * gradients to ||r|| <= tol ||b|| (free beads with no path to an electrode
 * keep V = 0 and carry no current).  Outputs:
 *   V_dev[n]  potentials; I_dev[n]  Eq. 15, I_i = 1/2 sum_j G_ij |V_i - V_j|
 *   (device, caller-owned, FP64);
 *   out->I_tot   the current leaving the source electrode,
 *   out->I_ref   dV / (x_snk - x_src): Eq. 16 with kappa_0 A = 1, the current
 *                of an ideal straight chain of beads across the gap,
 *   out->kappa   I_tot / I_ref (Eq. 18 for one deposit),
 *   out->edges, n_source, n_sink, max_degree, iterations, rel_residual.
 * pos_dev: [n][3] bead positions (device, FP64).  n <= LB_NET_MAX_BEADS; at
 * most LB_NET_MAX_DEG neighbours per bead (LB_EINVAL otherwise, after the
 * outputs are written).  LB_EUNSTABLE if the residual is still above tol
 * after max_iter iterations (outputs written).
 * workspace_dev: device scratch of at least lb_kirchhoff_workspace_bytes(n)
 * bytes, 256-byte aligned, caller-owned (LB_EINVAL if null, misaligned or
 * short while n > 0); nothing in it needs to be initialised and its contents
 * mean nothing after the call.  Allocates nothing; enqueued on `stream`,
 * then synchronises it to return the scalars.
 */
#define LB_NET_MAX_BEADS 65536
#define LB_NET_MAX_DEG 64
typedef struct {
    double r_c, x_src, x_snk, dV, tol;
    int32_t max_iter;
} lb_kirchhoff_spec;
typedef struct {
    double I_tot, I_ref, kappa, rel_residual;
    int32_t iterations, edges, n_source, n_sink, max_degree;
} lb_kirchhoff_out;
size_t lb_kirchhoff_workspace_bytes(int32_t n);
int lb_kirchhoff(const double *pos_dev, int32_t n, const lb_kirchhoff_spec *spec, double *V_dev, double *I_dev,
                 void *workspace_dev, size_t workspace_bytes, lb_kirchhoff_out *out, hipStream_t stream);

/*
 * lb_kirchhoff without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, outputs, errors and
 * synchronisation as lb_kirchhoff; the workspace is a fixed device array of
 * lb_kirchhoff_workspace_bytes(LB_NET_NOALLOC_MAX_BEADS) bytes (about 6.7 MB)
 * that each GPU holds from the first call until the process ends.  n above
 * LB_NET_NOALLOC_MAX_BEADS returns LB_EINVAL.  The stream must belong to the
 * current device.  Every call on one GPU uses that GPU's one array: calls
 * that overlap on one GPU (other streams, other host threads) race and give
 * undefined results.  The kernels write every scratch word before reading
 * it, so the previous call's contents do not matter.
 */
#define LB_NET_NOALLOC_MAX_BEADS 8192
int lb_kirchhoff_noalloc(const double *pos_dev, int32_t n, const lb_kirchhoff_spec *spec, double *V_dev,
                         double *I_dev, lb_kirchhoff_out *out, hipStream_t stream);

/* Beads of the rods for the network and the deposit profiles: nb = max(2,
 * floor(2 h / bead_spacing + 1/2) + 1) <= 64 beads per rod evenly along its
 * axis segment (half-length h = L/2 - R) about the stored centre, rod after
 * rod, into pos_dev [n_rods * nb][3] (device, caller-owned, capacity `cap`
 * beads).  *n_out = n_rods * nb (also when pos_dev is null or too small,
 * which then returns LB_EINVAL).  Enqueued on `stream`. */
int lb_rod_beads(lb_ctx *ctx, double bead_spacing, double *pos_dev, int32_t cap, int32_t *n_out, hipStream_t stream);

/* Tile shape of the fused step: 64 x tile_y columns, rows_per_thread rows per
 * thread, zchunk planes marched per work-group. */
typedef struct {
    int32_t tile_y, rows_per_thread, zchunk;
    double us_per_step;   /* measured by lb_autotune (0 when set by hand) */
} lb_tile;

/* Switch the tile shape of later steps (same rules as lb_params).  The
 * reservoir ledger is carried over exactly.  Asynchronous. */
int lb_set_tiles(lb_ctx *ctx, const lb_tile *tile, hipStream_t stream);

/* Time every supported tile shape for trial_steps >= 1 steps each (HIP events
 * on the stream), keep the fastest and return it in *best.  The trial steps
 * are real steps of the simulation (the state advances by n_shapes *
 * trial_steps steps).  Synchronises. */
int lb_autotune(lb_ctx *ctx, int32_t trial_steps, hipStream_t stream, lb_tile *best);

/*
 * Batches (many lattices per launch).  A batch advances n >= 1 lattices that
 * were each set up with lb_init (any sizes, parameters, rod counts and tile
 * shapes; one precision) with shared launches: one fused-step launch per
 * tile class walks a device work list of (lattice, tile) entries with a
 * parameter record per lattice, and each rod pass covers the rods of every
 * lattice.  Results are identical to stepping each lattice alone with
 * lb_step and lb_rods_step.  While a batch exists its lattices must be
 * stepped only through it (lb_batch_step fails with LB_EINVAL otherwise);
 * observables, export and rod reads work as usual.  The batch keeps its
 * records in a caller-owned device workspace of lb_batch_workspace_bytes()
 * bytes, which must outlive it.
 */
typedef struct lb_batch lb_batch;
size_t lb_batch_workspace_bytes(lb_ctx *const *ctxs, int32_t n); /* 0 on bad input */
/* Synchronises (uploads the work lists and records). */
int lb_batch_create(lb_ctx *const *ctxs, int32_t n, void *workspace_dev, hipStream_t stream, lb_batch **out);
/* nsteps steps of every lattice: the fused fluid step, then (with_rods != 0)
 * the rod update.  use_graph != 0: pairs of steps run as one HIP graph,
 * captured on first use on a stream of the batch's own and replayed on
 * `stream` (the graph holds no memset or memcpy nodes).  Asynchronous. */
int lb_batch_step(lb_batch *b, int32_t nsteps, int32_t with_rods, int32_t use_graph, hipStream_t stream);
int lb_batch_destroy(lb_batch *b);

/*
 * Learned surrogate (a 3-D convolutional U-Net advancing coarse-grained
 * fields; the paper has none).  A coarse canvas is [D][H][W][8]
 * channels-last: rho_A, rho_B, u_x, u_y, u_z, rod volume fraction, domain
 * mask (1 inside the lattice), fluid fraction (fluid nodes / 8).  Densities
 * are means over the fluid nodes of each 2 x 2 x 2 block; u is the block's
 * physical velocity sum (j + F/2) / sum rho over those nodes (Shan-Chen force F,
 * the velocity the method reports), read off the stored post-collision state
 * as j* - F/2.  The lattice occupies cells [0, n/2) per axis (n even, n/2 <=
 * canvas size); cells outside hold gas (0.03, 1), zero velocity, mask 0 and
 * fluid fraction 0.
 *
 * lb_sur_restrict : canvas of the current state into coarse_f32 and/or
 *                   coarse_bf16 (device, caller-owned, nullable one of them).
 * lb_sur_lift     : prolongation of channels 0..4 of coarse (device FP32
 *                   canvas) to every fluid node: trilinear from coarse
 *                   coordinate x/2 - 1/4 over the corner cells holding fluid,
 *                   renormalised (else the mean of the fluid-holding cells of
 *                   the 4 x 4 x 4 block around them, else gas at rest),
 *                   each rho_k clamped at 0 and a speed above 0.15 scaled
 *                   down to 0.15 (a prediction can leave the states the
 *                   lattice takes); then
 *                   the collision output of those fields becomes the current
 *                   state: f_k = f^eq(rho_k, u - F/(2 rho) + tau_k F_k / rho_k)
 *                   (Eq. 2) with F the force of the lifted densities (no
 *                   F/(2 rho) shift where rho vanishes); wall and
 *                   rod bounce-back slots are refreshed.
 * Both asynchronous; LB_EINVAL on null pointers or a lattice that does not
 * fit.  Both use the context's other population buffer as scratch (it holds
 * no state between steps).
 */
int lb_sur_restrict(lb_ctx *ctx, int32_t D, int32_t H, int32_t W, float *coarse_f32, void *coarse_bf16,
                    hipStream_t stream);
int lb_sur_lift(lb_ctx *ctx, const float *coarse_f32, int32_t D, int32_t H, int32_t W, hipStream_t stream);
/* Rods over a surrogate jump of `steps` lattice steps: each centre moves by
 * steps x the mean of the coarse velocities of coarse_now and coarse_next
 * (trilinear at the centre, from coarse coordinate x/2 - 1/4; kept one node
 * off closed end planes), V takes that mean, orientation and angular momentum
 * are kept.  A rods-only relaxation then removes the overlaps the move made:
 * Jacobi sweeps move both rods of a pair whose axis segments are closer than
 * rod_d0 apart by half the deficit along the closest-point direction (and a
 * rod whose axis end is closer than rod_d0_wall to the wall up), until no
 * deficit exceeds 1e-6 or 200 sweeps are done.  The rods are then re-placed
 * (rod nodes recomputed, no mass booked).  Call before lb_sur_lift, which
 * fills the vacated nodes.  Asynchronous. */
int lb_sur_jump_rods(lb_ctx *ctx, const float *coarse_now, const float *coarse_next, int32_t D, int32_t H, int32_t W,
                     double steps, hipStream_t stream);
/* Rods over a surrogate jump from their own recent motion (the alternative to
 * lb_sur_jump_rods): each centre continues `factor` times its minimum-image
 * displacement since x_prev, the device array [n_rods][3] (FP64, x y z) of the
 * centres one interval earlier (owned by the caller, read before the call
 * returns its work to the stream); kept one node off closed end planes.
 * Velocity, orientation and angular momentum are kept; the same rods-only
 * relaxation and re-placement as lb_sur_jump_rods follow.  Call before
 * lb_sur_lift.  LB_EINVAL for a null pointer or a non-finite factor; a lattice
 * without rods returns at once.  Asynchronous. */
int lb_sur_drift_rods(lb_ctx *ctx, const double *x_prev, double factor, hipStream_t stream);

/*
 * 3-D convolution, 3 x 3 x 3 taps, zero padding, channels-last BF16 tensors
 * [D][H][W][C] on the device, FP32 accumulation on the matrix cores:
 *   y[p, o] = b[o] + sum_{t, c} x[p + o_t, c] w[t, c, o], then ReLU if relu.
 * The input is the concatenation of x1 (channels [0, c1); at half resolution
 * and read through nearest-neighbour upsampling when up1 != 0) and x2
 * (channels [c1, c1 + c2), full resolution; c2 = 0 for none).  w: BF16
 * [27][c1 + c2][cout], tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1); wt: the
 * same weights packed [cout][27][c1 + c2] (lb_conv_pack_weights), read by the
 * forward only; b: FP32 [cout] or null; outputs y (BF16) and/or yf (FP32)
 * [D][H][W][cout]; acc: nullable FP32 scratch [D][H][W][cout] (forward
 * only; with it a layer of few output tiles splits its K range over more
 * work-groups, adding partial sums with atomics, so the summation order
 * varies).  c1, c2, cout: multiples of 8; D, H, W even when up1;
 * D H W max(c1 + c2, cout) < 2^31.  Asynchronous; LB_EINVAL on bad shapes or
 * null pointers.
 */
typedef struct {
    const void *x1;
    int32_t c1, up1;
    const void *x2;
    int32_t c2;
    const void *w;
    const void *wt;
    const float *b;
    void *y;
    float *yf;
    float *acc;
    int32_t D, H, W, cout, relu;
} lb_conv;
int lb_conv3d_forward(const lb_conv *conv, hipStream_t stream);
/* wt [cout][27][cin] = w [27][cin][cout] (BF16, device). */
int lb_conv_pack_weights(const void *w, int32_t cin, int32_t cout, void *wt, hipStream_t stream);
/* g = BF16(dy) masked by y > 0 when relu (dy FP32, y BF16, n elements): the
 * gradient at a convolution's pre-activation, the operand of both backward
 * passes below. */
int lb_relu_grad(const float *dy, const void *y, int64_t n, int32_t relu, void *g, hipStream_t stream);
/* dx [D][H][W][c1 + c2] FP32 (overwritten) = the input gradient for the
 * pre-activation gradient g [D][H][W][cout] BF16 (lb_relu_grad).  Layers of
 * few output tiles split K and add into dx with atomics (order varies). */
int lb_conv3d_backward_data(const lb_conv *conv, const void *g, float *dx, hipStream_t stream);
/* dw [27][c1 + c2][cout] and db [cout] (nullable) FP32 += the parameter
 * gradients for g (accumulated with atomics, so the summation order varies). */
int lb_conv3d_backward_weights(const lb_conv *conv, const void *g, float *dw, float *db, hipStream_t stream);
/* 2 x 2 x 2 average pooling of BF16 x [D][H][W][C] into y [D/2][H/2][W/2][C]. */
int lb_pool2(const void *x, int32_t D, int32_t H, int32_t W, int32_t C, void *y, hipStream_t stream);
/* g[p, c] = gc[parent(p), c] / 8 (+ skip[p * skip_stride + skip_off + c] when
 * skip is not null): the gradient through pooling plus a skip connection. */
int lb_pool2_backward(const float *gc, const float *skip, int32_t skip_stride, int32_t skip_off, int32_t D, int32_t H,
                      int32_t W, int32_t C, float *g, hipStream_t stream);
/* gc[q, c] = sum of g[p * stride + c] over the 8 children p of q: the gradient
 * through nearest-neighbour upsampling. */
int lb_up2_backward(const float *g, int32_t stride, int32_t C, int32_t D, int32_t H, int32_t W, float *gc,
                    hipStream_t stream);
int lb_fill_f32(float *p, int64_t n, float value, hipStream_t stream);        /* graph-safe clear */

/*
 * The whole surrogate network in one call each way (the learned surrogate: a
 * 3-D convolutional encoder-decoder on the coarse canvas).  nlev levels
 * (2..4) of ch[l] channels: per level two 3x3x3 ReLU convolutions, 2x2x2
 * average pooling down; on the way up nearest-neighbour upsampling
 * concatenated with the level's skip, two ReLU convolutions; a final linear
 * 3x3x3 convolution to cout channels.  Layers are numbered in forward order:
 * enc0a, enc0b, ..., enc{nlev-1}b, dec{nlev-2}a, dec{nlev-2}b, ..., dec0b,
 * out (4 nlev - 1 layers).  All pointers are device buffers owned by the
 * caller, channels-last [D][H][W][C] per level l of P_l = (D H W) / 8^l
 * cells:
 *   p, g     FP32 parameters and gradients (layer L: weights [27][cin][cout]
 *            at off_w[L], biases [cout] at off_b[L], element offsets, 4-byte
 *            aligned blocks of 16 bytes);
 *   pb, pt   BF16 weights, and the same packed [cout][27][cin] for the
 *            forward (lb_conv_pack_weights), at the same offsets;
 *   act[L]   BF16 outputs of the hidden layers L < 4 nlev - 2, P_l x ch[l];
 *   pooled   BF16 pooled maps, level l: P_{l+1} x ch[l];
 *   out      FP32 network output [P_0][cout];
 *   gA, gB   FP32 gradient scratch per level, P_l x max(ch[l] + ch[l+1],
 *            cin, 2 ch[nlev-1]) and P_l x max(ch) elements;
 *   gcat     FP32 per level l < nlev - 1, P_l x (ch[l] + ch[l+1]) elements;
 *   gm       BF16 scratch of the largest layer output, P_l x cout;
 *   acc      FP32 split-K scratch of the coarse levels (largest layer output
 *            of levels >= 1).
 * cin and the channel counts are multiples of 8; D, H, W divisible by
 * 2^(nlev-1).  lb_sur_forward(x) writes act, pooled and out for the BF16
 * input x [P_0][cin]; lb_sur_backward(x, gout) adds to g the parameter
 * gradients for dloss/dout = gout [P_0][cout] (FP32) of the forward of the
 * same x, whose activations it reads.  Asynchronous; LB_EINVAL on bad
 * shapes or null pointers.
 */
#define LB_UNET_MAXLEV 4
#define LB_UNET_MAXLAYER (4 * LB_UNET_MAXLEV - 1)
typedef struct {
    int32_t D, H, W, nlev, cin, cout;
    int32_t ch[LB_UNET_MAXLEV];
    float *p, *g;
    void *pb, *pt;
    int64_t off_w[LB_UNET_MAXLAYER], off_b[LB_UNET_MAXLAYER];
    void *act[LB_UNET_MAXLAYER];
    void *pooled[LB_UNET_MAXLEV];
    float *out;
    float *gA[LB_UNET_MAXLEV], *gB[LB_UNET_MAXLEV], *gcat[LB_UNET_MAXLEV];
    void *gm;
    float *acc;
} lb_unet;
int lb_sur_forward(const lb_unet *net, const void *x, hipStream_t stream);
int lb_sur_backward(const lb_unet *net, const void *x, const float *gout, hipStream_t stream);
int lb_to_bf16(const float *x, int64_t n, void *y, hipStream_t stream);       /* round to nearest even */
/* Network input from an FP32 canvas of P cells: y[:, c] = BF16((x[:, c] -
 * shift[c]) * gain[c]) (shift, gain: host, 8 finite values each). */
int lb_sur_normalize(const float *x, int64_t P, const float *shift, const float *gain, void *y, hipStream_t stream);
/* Network prediction on P canvas cells: pred[:, c] = xin[:, c] + scale[c] *
 * out[:, c] for c < 6 (residual; scale: host, 6 positive values, null = 1),
 * channels 6, 7 copied from xin; into pred (FP32) and/or pred_bf16. */
int lb_sur_residual(const float *out, const float *xin, int64_t P, const float *scale, float *pred, void *pred_bf16,
                    hipStream_t stream);
/* Surrogate loss over P cells of [P][8] FP32 tensors in channel-normalised
 * units: pred = xin[0:6] + scale * out[0:6], e = (pred - tgt) / scale, mask =
 * xin[6]; loss = masked mean of e^2 over the six channels + lam * (relative
 * rho_A mass error)^2.  grad (nullable) [P][8] receives dloss/dout.  scratch:
 * device, lb_sur_loss_scratch_bytes() bytes.  result_host (nullable; the call
 * then synchronises): sum mask, sum mask tgt_A, relative mass error, loss. */
size_t lb_sur_loss_scratch_bytes(void);
int lb_sur_loss(const float *out, const float *xin, const float *tgt, int64_t P, const float *scale, double lam,
                float *grad, void *scratch, double *result_host, hipStream_t stream);
/* Per-channel sums over P cells of mask * (y - x)^2 (channels 0..5) and of the
 * mask (xin channel 6) into result_host[7]; the scratch of lb_sur_loss.
 * Synchronises. */
int lb_sur_moments(const float *x, const float *y, int64_t P, void *scratch, double *result_host, hipStream_t stream);
/* Adam (Kingma and Ba) with bias correction on n FP32 master parameters p
 * with moments m, v; p_bf16 (nullable) receives the rounded copy.  step >= 1. */
int lb_adam(float *p, const float *g, float *m, float *v, void *p_bf16, int64_t n, int32_t step, double lr, double b1,
            double b2, double eps, hipStream_t stream);

/* Index (0 or 1) of the buffer holding the current state. */
int lb_current_buffer(const lb_ctx *ctx);

/* Destroy the host context (device buffers stay with the caller). */
int lb_destroy(lb_ctx *ctx);

/* Thread-local text of the last error. */
const char *lb_last_error(void);

/* sizeof of lb_params, lb_buffers, lb_obs, lb_droplet, lb_deposit_spec,
 * lb_graph, lb_conv, lb_kirchhoff_spec, lb_kirchhoff_out and lb_unet into
 * out[0..9], so a binding can verify its mirrors of the structs.  Never
 * fails. */
void lb_abi_sizes(size_t out[10]);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
