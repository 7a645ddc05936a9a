"""Pins of the observables oracle: closed forms, exact special cases, brute force."""
import numpy as np
import pytest

from oracle import lbm
from oracle import observables as O
from oracle import rods as R

RNG = np.random.default_rng(5150)


def _cap_rho(shape, centre, radius):
    """Two-phase field whose colour is exactly C = radius - |x - centre| (rho_A + rho_B = 1)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    C = radius - d
    rho = np.stack([(1 + C) / 2, (1 - C) / 2])
    mat = np.zeros(shape, np.uint8)
    mat[0] = 3
    rho[:, 0] = 0.0
    return rho, mat


def test_spherical_cap_height_footprint_and_angle():
    """Apex height is exact (C linear along the centre column); footprint and
    the spherical-cap angle match the geometry of the sphere."""
    shape = (40, 64, 80)
    for zc, Rs in ((6.3, 20.0), (-4.7, 25.0)):
        centre = (40.0, 32.0, zc)
        rho, mat = _cap_rho(shape, centre, Rs)
        d = O.droplet_shape(rho, mat, 40.0, 32.0)
        # apex: the C = 0 crossing of the centre column at zc + Rs, above the wall at 1/2
        assert d.height == pytest.approx(zc + Rs - 0.5, abs=1e-12)
        # footprint on the plane z = 1 (linear interpolation of a circle: small error)
        r1 = np.sqrt(Rs ** 2 - (1 - zc) ** 2)
        assert d.r_x == pytest.approx(r1, abs=0.02) and d.r_y == pytest.approx(r1, abs=0.02)
        # spherical-cap identity h / r = tan(theta / 2) against the geometric angle at the wall
        theta_geo = np.arccos(-(zc - 0.5) / Rs)
        assert d.theta_x == pytest.approx(theta_geo, abs=np.radians(1.0))
        assert d.theta_x == pytest.approx(2 * np.arctan(d.height / d.r_x), rel=1e-14)


def test_dry_and_flat_film_cases():
    shape = (12, 10, 14)
    rho = np.zeros((2,) + shape)
    rho[1] = 1.0
    mat = np.zeros(shape, np.uint8)
    mat[0] = 3
    d = O.droplet_shape(rho, mat, 6.5, 4.5)
    assert d.height == 0 and d.r_x == 0 and d.r_y == 0 and d.wet_nodes == 0
    # flat film of 4 wet planes with a sharp top: crossing half-way to the next plane
    rho[0, 1:5] = 1.0
    rho[1, 1:5] = 0.0
    d = O.droplet_shape(rho, mat, 6.5, 4.5)
    assert d.height == pytest.approx(4.0)  # z* = 4, crossing 4.5, wall at 0.5
    assert d.wet_nodes == 4 * 10 * 14
    # the film spans the periodic row: the run ends at the array ends (half a node out)
    assert d.r_x == pytest.approx(7.0) and d.r_y == pytest.approx(5.0)


def _rods_along(e, n, box, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, 3)) * np.array(box, float)
    q = np.tile(_quat_to(e), (n, 1))
    return X, q


def _quat_to(e):
    e = np.asarray(e, float) / np.linalg.norm(e)
    if e[2] < -1 + 1e-12:
        return np.array([0.0, 1.0, 0.0, 0.0])
    q = np.array([1.0 + e[2], -e[1], e[0], 0.0])
    return q / np.linalg.norm(q)


def test_nematic_order_special_cases():
    """S_x = 1 for axial, -1 for transverse, 0 for 45-degree segments (exact)."""
    box = (96, 48, 32)
    spec = O.DepositSpec(n_bins_x=12, n_bins_y=6, xc=47.5, yc=23.5, strip_x=60, strip_y=30)
    for e, want in (((1, 0, 0), 1.0), ((0, 1, 0), -1.0), ((0, 0, 1), -1.0), ((1, 1, 0), 0.0)):
        X, q = _rods_along(e, 40, box, 11)
        gx, Sx, Nx, gy, Sy, Ny = O.deposit_profiles(X, q, 10.0, box, spec)
        assert np.all(np.abs(Sx[Nx > 0] - want) < 1e-12) and np.all(Sx[Nx == 0] == 0)
        assert np.all(np.abs(Sy[Ny > 0] - want) < 1e-12)


def test_density_profile_mean_is_one_and_counts_beads():
    box = (96, 48, 32)
    spec = O.DepositSpec(n_bins_x=16, n_bins_y=8, xc=47.5, yc=23.5, strip_x=1e9, strip_y=1e9)
    n = 25
    X = RNG.uniform(0, 1, (n, 3)) * np.array(box, float)
    q = RNG.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    gx, Sx, Nx, gy, Sy, Ny = O.deposit_profiles(X, q, 10.0, box, spec)
    # Eq. 14 with equal bins: the bin mean of g is exactly one
    assert gx.mean() == pytest.approx(1.0, abs=1e-14) and gy.mean() == pytest.approx(1.0, abs=1e-14)
    # with an unbounded strip every bead and segment is binned once
    nb = 11  # 2 half / spacing + 1
    assert Nx.sum() == n * (nb - 1) and Ny.sum() == n * (nb - 1)
    # bead counts: reconstruct directly from the bead coordinates
    cnt = np.zeros(16)
    for r in range(n):
        B, _ = O.beads(X[r], q[r], 10.0, 2.0)
        for p in B:
            cnt[min(int(np.floor((p[0] % 96) * 16 / 96)), 15)] += 1
    assert np.allclose(gx, cnt / cnt.mean(), rtol=1e-15)


def test_strip_selects_central_band():
    """Beads outside |y - yc| <= strip_y / 2 do not enter the axial profile."""
    box = (64, 64, 32)
    X = np.array([[20.0, 32.0, 10.0], [40.0, 5.0, 10.0]])
    q = np.tile(_quat_to((1, 0, 0)), (2, 1))
    spec = O.DepositSpec(n_bins_x=8, n_bins_y=8, xc=31.5, yc=31.5, strip_x=20, strip_y=10)
    gx, Sx, Nx, gy, Sy, Ny = O.deposit_profiles(X, q, 6.0, box, spec)
    assert Nx.sum() == 6  # 7 beads, 6 segments of the first rod only
    # first rod spans x in [14, 26]: bins 1..3 of width 8
    assert set(np.nonzero(Nx)[0]) <= {1, 2, 3}


def test_contact_graph_chain_and_brute_force():
    box = (200, 64, 64)
    half = 10.0
    qx = _quat_to((1, 0, 0))
    # a chain of rods along x with end gaps of 4 (< 5.25): one cluster spanning
    X = np.array([[15.0 + 24.0 * i, 32.0, 20.0] for i in range(7)])
    Q = np.tile(qx, (7, 1))
    g = O.contact_graph(X, Q, half, box, (True, True, False), 5.25, 10.0, 150.0)
    assert g.edges == 6 and g.largest == 7 and g.spanning
    # widen one gap to 6: two clusters, no spanning
    X2 = X.copy()
    X2[4:, 0] += 2.0
    g2 = O.contact_graph(X2, Q, half, box, (True, True, False), 5.25, 10.0, 150.0)
    assert g2.edges == 5 and g2.largest == 4 and not g2.spanning
    assert len(set(g2.labels.tolist())) == 2
    # random rods: edges agree with a dense-sampling brute force away from the cutoff
    n = 30
    X3 = RNG.uniform(0, 1, (n, 3)) * np.array([60.0, 60.0, 40.0])
    Q3 = RNG.normal(size=(n, 4))
    Q3 /= np.linalg.norm(Q3, axis=1, keepdims=True)
    g3 = O.contact_graph(X3, Q3, half, (60, 60, 40), (False, False, False), 5.25, 0.0, 1e9)
    s = np.linspace(-half, half, 801)
    found = set(g3.pairs)
    checked = 0
    for a in range(n):
        A = X3[a] + s[:, None] * R.axis(Q3[a])[None]
        for b in range(a + 1, n):
            B = X3[b] + s[:, None] * R.axis(Q3[b])[None]
            d = np.sqrt(((A[:, None] - B[None]) ** 2).sum(-1)).min()
            # sampling overestimates the distance by at most one sampling step
            if abs(d - 5.25) < 0.03:
                continue
            checked += 1
            assert ((a, b) in found) == (d < 5.25)
    assert checked > 400 and len(found) > 5


def test_rod_column_map():
    mat = np.zeros((5, 4, 6), np.uint8)
    mat[1:4, 2, 3] = lbm.ROD
    mat[2, 0, 0] = lbm.ROD
    m = O.rod_column_map(mat)
    assert m[2, 3] == 3 and m[0, 0] == 1 and m.sum() == 4


# --------------------------------------------------------------------------
# ensemble profiles: runs and mirror images (the angle brackets of Eqs. 13-14)
# --------------------------------------------------------------------------
def _runs(seed, sizes):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        X = np.c_[rng.uniform(20, 76, n), rng.uniform(10, 38, n), rng.uniform(2, 4, n)]
        Q = [O._quat_of_axis(e) for e in rng.normal(size=(n, 3))]
        out.append((X, Q))
    return out


ESPEC = dict(n_bins_x=12, n_bins_y=6, xc=47.5, yc=23.5, strip_x=60, strip_y=30)


def test_ensemble_without_mirror_is_the_mean_of_the_runs():
    spec = O.DepositSpec(**ESPEC)
    runs = _runs(11, (30, 25, 7))
    e = O.ensemble_profiles(runs, 10.0, (96, 48, 20), spec, mirror=False)
    single = [O.deposit_profiles(X, Q, 10.0, (96, 48, 20), spec) for X, Q in runs]
    for d, (gi, si, ni) in enumerate(((0, 1, 2), (3, 4, 5))):
        assert np.allclose(e[gi], np.mean([p[gi] for p in single], axis=0), rtol=1e-15, atol=1e-15)
        assert np.array_equal(e[ni], np.sum([p[ni] for p in single], axis=0))
        # S: mean over the runs that have segments in the bin, by hand
        for b in range(len(e[si])):
            vals = [p[si][b] for p in single if p[ni][b] > 0]
            assert e[si][b] == pytest.approx(np.mean(vals) if vals else 0.0, abs=1e-15)
    assert e[0].mean() == pytest.approx(1.0, rel=1e-14)


def test_ensemble_with_mirror_images_is_symmetric():
    """The four images of a run give the same ensemble as the four images of
    its mirrored copy; a run placed symmetrically about the centre gives its
    own profile; an axial rod pair mirrored in x fills the mirror bins."""
    spec = O.DepositSpec(**ESPEC)
    box = (96, 48, 20)
    (X, Q), = _runs(12, (40,))
    Xm, Em = O.mirror_rods(X, Q, spec.xc, spec.yc, 1, 1)
    a = O.ensemble_profiles([(X, Q)], 10.0, box, spec)
    b = O.ensemble_profiles([(Xm, [O._quat_of_axis(e) for e in Em])], 10.0, box, spec)
    for u, v in zip(a, b):
        assert np.abs(u - v).max() < 1e-12
    # a rod along x at (xc - 20, yc) and its mirror at (xc + 20, yc): already symmetric
    qx = O._quat_of_axis([1.0, 0.0, 0.0])
    sym = (np.array([[spec.xc - 20.0, spec.yc, 3.0], [spec.xc + 20.0, spec.yc, 3.0]]), [qx, qx])
    e = O.ensemble_profiles([sym], 10.0, box, spec)
    p = O.deposit_profiles(*sym, 10.0, box, spec)
    assert np.allclose(e[0], p[0]) and np.allclose(e[1], p[1])
    # one rod only: its x-mirror image puts beads in the mirrored bins
    one = (sym[0][:1], sym[1][:1])
    e1 = O.ensemble_profiles([one], 10.0, box, spec)
    assert np.allclose(e1[0], e[0])
