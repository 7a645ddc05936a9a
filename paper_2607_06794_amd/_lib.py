"""ctypes binding of liblbm.so (the C ABI in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm.so")

LB_OK, LB_EINVAL, LB_ENOTSUP, LB_EHIP, LB_EUNSTABLE, LB_EPLACE = 0, -1, -2, -3, -4, 1
LB_F64, LB_F32, LB_F16DEV, LB_BF16DEV = 0, 1, 2, 3
LB_NMAT = 9
LB_MODEL_SC, LB_MODEL_CG = 0, 1
LB_MAX_RODS = 512
LB_FIL_MAX_BEADS = 4096
LB_NET_NOALLOC_MAX_BEADS = 8192  # include/lbm.h

# Every exported symbol declared in include/lbm.h
EXPORTS = (
    "lb_pop_stride",
    "lb_pop_bytes",
    "lb_workspace_bytes",
    "lb_init",
    "lb_step",
    "lb_observables",
    "lb_export",
    "lb_current_buffer",
    "lb_destroy",
    "lb_last_error",
    "lb_abi_sizes",
    "lb_set_tiles",
    "lb_autotune",
    "lb_rods_step",
    "lb_rods_get",
    "lb_fil_set",
    "lb_fil_step",
    "lb_fil_get",
    "lb_droplet_shape",
    "lb_deposit",
    "lb_rod_map",
    "lb_kirchhoff",
    "lb_deposit_ensemble",
    "lb_sur_forward",
    "lb_sur_backward",
    "lb_kirchhoff_workspace_bytes",
    "lb_kirchhoff_noalloc",
    "lb_rod_beads",
    "lb_batch_workspace_bytes",
    "lb_batch_create",
    "lb_batch_step",
    "lb_batch_destroy",
    "lb_sur_restrict",
    "lb_sur_lift",
    "lb_sur_jump_rods",
    "lb_sur_drift_rods",
    "lb_conv3d_forward",
    "lb_conv3d_backward_data",
    "lb_conv3d_backward_weights",
    "lb_conv_pack_weights",
    "lb_relu_grad",
    "lb_pressure",
    "lb_sur_normalize",
    "lb_pool2",
    "lb_pool2_backward",
    "lb_up2_backward",
    "lb_fill_f32",
    "lb_to_bf16",
    "lb_sur_residual",
    "lb_sur_moments",
    "lb_sur_loss_scratch_bytes",
    "lb_sur_loss",
    "lb_adam",
)


class LbParams(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int32),
        ("ny", ct.c_int32),
        ("nz", ct.c_int32),
        ("periodic", ct.c_int32 * 3),
        ("prec", ct.c_int32),
        ("tau", ct.c_double * 2),
        ("G", ct.c_double),
        ("body_force", ct.c_double * 3),
        ("psi_solid", (ct.c_double * 2) * LB_NMAT),
        ("evap_on", ct.c_int32),
        ("rho_top", ct.c_double * 2),
        ("rho_ref", ct.c_double * 2),
        ("n_rods", ct.c_int32),
        ("n_sub", ct.c_int32),
        ("rod_length", ct.c_double),
        ("rod_radius", ct.c_double),
        ("rod_rho", ct.c_double),
        ("eps_att", ct.c_double),
        ("eps_rep", ct.c_double),
        ("rod_d0", ct.c_double),
        ("rod_rcut", ct.c_double),
        ("eps_wall", ct.c_double),
        ("rod_d0_wall", ct.c_double),
        ("wall_on", ct.c_int32),
        ("wall_z", ct.c_double),
        ("tile_y", ct.c_int32),
        ("rows_per_thread", ct.c_int32),
        ("zchunk", ct.c_int32),
        ("sink_on", ct.c_int32),
        ("sink_J0", ct.c_double),
        ("sink_K", ct.c_double),
        ("sink_h0", ct.c_double),
        ("model", ct.c_int32),
        ("cg_sigma", ct.c_double),
        ("cg_beta", ct.c_double),
        ("cg_grad_eps", ct.c_double),
        ("cg_theta", ct.c_double * LB_NMAT),
        ("round_stochastic", ct.c_int32),
        ("sr_seed", ct.c_uint32),
        ("n_fil", ct.c_int32),
        ("fil_beads", ct.c_int32),
        ("fil_k_s", ct.c_double),
        ("fil_R_m", ct.c_double),
        ("fil_eps", ct.c_double),
        ("fil_d0", ct.c_double),
        ("fil_k_b", ct.c_double),
        ("fil_eps_coh", ct.c_double),
        ("fil_r_cut", ct.c_double),
        ("fil_eps_s", ct.c_double),
        ("fil_sigma_s", ct.c_double),
        ("fil_r_cut_s", ct.c_double),
        ("fil_mu", ct.c_double),
        ("fil_gamma", ct.c_double),
        ("fil_kappa_s", ct.c_double),
        ("fil_skin", ct.c_double),
    ]


class LbBuffers(ct.Structure):
    _fields_ = [("f", ct.c_void_p * 2), ("workspace", ct.c_void_p)]


class LbObs(ct.Structure):
    _fields_ = [
        ("step", ct.c_int64),
        ("mass", ct.c_double * 2),
        ("ledger", ct.c_double * 2),
        ("momentum", ct.c_double * 3),
        ("max_speed", ct.c_double),
        ("kinetic", ct.c_double),
        ("fluid_nodes", ct.c_int64),
        ("status", ct.c_uint32),
        ("solid", ct.c_double * 2),
        ("rod_momentum", ct.c_double * 3),
    ]


class LbTile(ct.Structure):
    _fields_ = [
        ("tile_y", ct.c_int32),
        ("rows_per_thread", ct.c_int32),
        ("zchunk", ct.c_int32),
        ("us_per_step", ct.c_double),
    ]


class LbDroplet(ct.Structure):
    _fields_ = [
        ("height", ct.c_double),
        ("r_x", ct.c_double),
        ("r_y", ct.c_double),
        ("theta_x", ct.c_double),
        ("theta_y", ct.c_double),
        ("wet_nodes", ct.c_int64),
    ]


class LbDepositSpec(ct.Structure):
    _fields_ = [
        ("n_bins_x", ct.c_int32),
        ("n_bins_y", ct.c_int32),
        ("xc", ct.c_double),
        ("yc", ct.c_double),
        ("strip_x", ct.c_double),
        ("strip_y", ct.c_double),
        ("bead_spacing", ct.c_double),
        ("r_contact", ct.c_double),
        ("x_src", ct.c_double),
        ("x_snk", ct.c_double),
    ]


class LbGraph(ct.Structure):
    _fields_ = [
        ("n_rods", ct.c_int32),
        ("edges", ct.c_int32),
        ("largest", ct.c_int32),
        ("spanning", ct.c_int32),
    ]


class LbKirchhoffSpec(ct.Structure):
    _fields_ = [
        ("r_c", ct.c_double),
        ("x_src", ct.c_double),
        ("x_snk", ct.c_double),
        ("dV", ct.c_double),
        ("tol", ct.c_double),
        ("max_iter", ct.c_int32),
    ]


class LbKirchhoffOut(ct.Structure):
    _fields_ = [
        ("I_tot", ct.c_double),
        ("I_ref", ct.c_double),
        ("kappa", ct.c_double),
        ("rel_residual", ct.c_double),
        ("iterations", ct.c_int32),
        ("edges", ct.c_int32),
        ("n_source", ct.c_int32),
        ("n_sink", ct.c_int32),
        ("max_degree", ct.c_int32),
    ]


class LbConv(ct.Structure):
    _fields_ = [
        ("x1", ct.c_void_p),
        ("c1", ct.c_int32),
        ("up1", ct.c_int32),
        ("x2", ct.c_void_p),
        ("c2", ct.c_int32),
        ("w", ct.c_void_p),
        ("wt", ct.c_void_p),
        ("b", ct.c_void_p),
        ("y", ct.c_void_p),
        ("yf", ct.c_void_p),
        ("acc", ct.c_void_p),
        ("D", ct.c_int32),
        ("H", ct.c_int32),
        ("W", ct.c_int32),
        ("cout", ct.c_int32),
        ("relu", ct.c_int32),
    ]


LB_UNET_MAXLEV = 4
LB_UNET_MAXLAYER = 4 * LB_UNET_MAXLEV - 1


class LbUnet(ct.Structure):
    _fields_ = [
        ("D", ct.c_int32), ("H", ct.c_int32), ("W", ct.c_int32), ("nlev", ct.c_int32), ("cin", ct.c_int32),
        ("cout", ct.c_int32),
        ("ch", ct.c_int32 * LB_UNET_MAXLEV),
        ("p", ct.c_void_p), ("g", ct.c_void_p), ("pb", ct.c_void_p), ("pt", ct.c_void_p),
        ("off_w", ct.c_int64 * LB_UNET_MAXLAYER), ("off_b", ct.c_int64 * LB_UNET_MAXLAYER),
        ("act", ct.c_void_p * LB_UNET_MAXLAYER),
        ("pooled", ct.c_void_p * LB_UNET_MAXLEV),
        ("out", ct.c_void_p),
        ("gA", ct.c_void_p * LB_UNET_MAXLEV), ("gB", ct.c_void_p * LB_UNET_MAXLEV), ("gcat", ct.c_void_p * LB_UNET_MAXLEV),
        ("gm", ct.c_void_p),
        ("acc", ct.c_void_p),
    ]


STRUCTS = ("LbParams", "LbBuffers", "LbObs", "LbDroplet", "LbDepositSpec", "LbGraph", "LbConv", "LbKirchhoffSpec",
           "LbKirchhoffOut", "LbUnet")


class LbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load liblbm.so (once) and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    # liblbm must bind to the same HIP runtime as PyTorch (which allocates the
    # device buffers and owns the streams); loading torch first makes the
    # dynamic loader resolve libamdhip64.so.7 to torch's copy
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first (python -m paper_2607_06794_amd.build); "
            "there is no CPU fallback"
        )
    lib = ct.CDLL(path)
    P = ct.POINTER
    lib.lb_pop_stride.argtypes = [P(LbParams)]
    lib.lb_pop_stride.restype = ct.c_int64
    lib.lb_pop_bytes.argtypes = [P(LbParams)]
    lib.lb_pop_bytes.restype = ct.c_size_t
    lib.lb_workspace_bytes.argtypes = [P(LbParams)]
    lib.lb_workspace_bytes.restype = ct.c_size_t
    lib.lb_init.argtypes = [P(LbParams), P(LbBuffers), ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                            P(ct.c_void_p)]
    lib.lb_init.restype = ct.c_int
    lib.lb_step.argtypes = [ct.c_void_p, ct.c_int32, ct.c_void_p]
    lib.lb_step.restype = ct.c_int
    lib.lb_observables.argtypes = [ct.c_void_p, P(LbObs), ct.c_void_p]
    lib.lb_observables.restype = ct.c_int
    lib.lb_export.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.lb_export.restype = ct.c_int
    lib.lb_current_buffer.argtypes = [ct.c_void_p]
    lib.lb_current_buffer.restype = ct.c_int
    lib.lb_destroy.argtypes = [ct.c_void_p]
    lib.lb_destroy.restype = ct.c_int
    lib.lb_last_error.argtypes = []
    lib.lb_last_error.restype = ct.c_char_p
    lib.lb_rods_step.argtypes = [ct.c_void_p, ct.c_void_p]
    lib.lb_rods_step.restype = ct.c_int
    lib.lb_rods_get.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.lb_rods_get.restype = ct.c_int
    lib.lb_fil_set.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.lb_fil_set.restype = ct.c_int
    lib.lb_fil_step.argtypes = [ct.c_void_p, ct.c_void_p]
    lib.lb_fil_step.restype = ct.c_int
    lib.lb_fil_get.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.lb_fil_get.restype = ct.c_int
    lib.lb_set_tiles.argtypes = [ct.c_void_p, P(LbTile), ct.c_void_p]
    lib.lb_set_tiles.restype = ct.c_int
    lib.lb_autotune.argtypes = [ct.c_void_p, ct.c_int32, ct.c_void_p, P(LbTile)]
    lib.lb_autotune.restype = ct.c_int
    lib.lb_droplet_shape.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, P(LbDroplet), ct.c_void_p]
    lib.lb_droplet_shape.restype = ct.c_int
    lib.lb_deposit.argtypes = [ct.c_void_p, P(LbDepositSpec)] + [ct.c_void_p] * 7 + [P(LbGraph), ct.c_void_p]
    lib.lb_deposit.restype = ct.c_int
    lib.lb_deposit_ensemble.argtypes = [ct.c_void_p, ct.c_int32, P(LbDepositSpec), ct.c_int32] + [ct.c_void_p] * 7
    lib.lb_deposit_ensemble.restype = ct.c_int
    lib.lb_sur_forward.argtypes = [P(LbUnet), ct.c_void_p, ct.c_void_p]
    lib.lb_sur_forward.restype = ct.c_int
    lib.lb_sur_backward.argtypes = [P(LbUnet), ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.lb_sur_backward.restype = ct.c_int
    lib.lb_rod_map.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.lb_rod_map.restype = ct.c_int
    lib.lb_kirchhoff.argtypes = [ct.c_void_p, ct.c_int32, P(LbKirchhoffSpec), ct.c_void_p, ct.c_void_p,
                                 ct.c_void_p, ct.c_size_t, P(LbKirchhoffOut), ct.c_void_p]
    lib.lb_kirchhoff.restype = ct.c_int
    lib.lb_kirchhoff_workspace_bytes.argtypes = [ct.c_int32]
    lib.lb_kirchhoff_workspace_bytes.restype = ct.c_size_t
    lib.lb_kirchhoff_noalloc.argtypes = [ct.c_void_p, ct.c_int32, P(LbKirchhoffSpec), ct.c_void_p, ct.c_void_p,
                                         P(LbKirchhoffOut), ct.c_void_p]
    lib.lb_kirchhoff_noalloc.restype = ct.c_int
    lib.lb_rod_beads.argtypes = [ct.c_void_p, ct.c_double, ct.c_void_p, ct.c_int32, P(ct.c_int32), ct.c_void_p]
    lib.lb_rod_beads.restype = ct.c_int
    lib.lb_batch_workspace_bytes.argtypes = [P(ct.c_void_p), ct.c_int32]
    lib.lb_batch_workspace_bytes.restype = ct.c_size_t
    lib.lb_batch_create.argtypes = [P(ct.c_void_p), ct.c_int32, ct.c_void_p, ct.c_void_p, P(ct.c_void_p)]
    lib.lb_batch_create.restype = ct.c_int
    lib.lb_batch_step.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p]
    lib.lb_batch_step.restype = ct.c_int
    lib.lb_batch_destroy.argtypes = [ct.c_void_p]
    lib.lb_batch_destroy.restype = ct.c_int
    V, I32, I64, D_ = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_double
    sigs = {
        "lb_sur_restrict": [V, I32, I32, I32, V, V, V],
        "lb_sur_lift": [V, V, I32, I32, I32, V],
        "lb_sur_jump_rods": [V, V, V, I32, I32, I32, D_, V],
        "lb_sur_drift_rods": [V, V, D_, V],
        "lb_conv3d_forward": [P(LbConv), V],
        "lb_conv3d_backward_data": [P(LbConv), V, V, V],
        "lb_conv3d_backward_weights": [P(LbConv), V, V, V, V],
        "lb_pool2": [V, I32, I32, I32, I32, V, V],
        "lb_conv_pack_weights": [V, I32, I32, V, V],
        "lb_relu_grad": [V, V, I64, I32, V, V],
        "lb_pressure": [V, V, I32, V, V],
        "lb_sur_normalize": [V, I64, V, V, V, V],
        "lb_pool2_backward": [V, V, I32, I32, I32, I32, I32, I32, V, V],
        "lb_up2_backward": [V, I32, I32, I32, I32, I32, V, V],
        "lb_fill_f32": [V, I64, ct.c_float, V],
        "lb_to_bf16": [V, I64, V, V],
        "lb_sur_loss": [V, V, V, I64, V, D_, V, V, V, V],
        "lb_sur_residual": [V, V, I64, V, V, V, V],
        "lb_sur_moments": [V, V, I64, V, V, V],
        "lb_adam": [V, V, V, V, V, I64, I32, D_, D_, D_, D_, V],
    }
    for name, args in sigs.items():
        getattr(lib, name).argtypes = args
        getattr(lib, name).restype = ct.c_int
    lib.lb_sur_loss_scratch_bytes.argtypes = []
    lib.lb_sur_loss_scratch_bytes.restype = ct.c_size_t
    lib.lb_abi_sizes.argtypes = [P(ct.c_size_t)]
    lib.lb_abi_sizes.restype = None
    sizes = (ct.c_size_t * len(STRUCTS))()
    lib.lb_abi_sizes(sizes)
    want = tuple(ct.sizeof(globals()[n]) for n in STRUCTS)
    if tuple(sizes) != want:
        raise RuntimeError(f"liblbm struct sizes {tuple(sizes)} differ from the binding's {want}")
    _lib = lib
    return lib


def check(rc: int, allow=(LB_OK,)):
    if rc not in allow:
        msg = load().lb_last_error()
        raise LbError(rc, msg.decode() if msg else "")
    return rc
