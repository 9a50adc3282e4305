"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, TOL_MEDIAN, make_sim, oracle_reference, rel_errors, stats, torch_dev
from paper_1003_3896_amd import inputs

pytestmark = pytest.mark.gpu


def _ragged_batch(seed=7, sizes=(1, 2, 3, 255, 256, 257, 700, 1000), field_every=3, eps=1e-3):
    cl = []
    for c, n in enumerate(sizes):
        p, v, m = inputs.plummer(n, seed * 100 + c, salpeter=(c % 2 == 1))
        fld = (c % field_every == 0)
        if fld:
            p, v = inputs.on_orbit(p, v)
        cl.append(inputs.single(p, v, m, eps, fld))
    return inputs.concat(cl)


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32c", "fp32", "fp32dl"])
def test_accel_single_cluster(prec):
    torch_dev()
    p, v, m = inputs.plummer(1000, 1234)
    b = inputs.single(p, v, m, 1e-3)
    sim = make_sim(b, prec)
    a = sim.accel().cpu().numpy()
    ref, scale = oracle_reference(b)
    err = rel_errors(a, ref, scale)
    print("\n[accel %s N=1000] %s" % (prec, stats(err)), flush=True)
    if prec in TOL:
        assert err.max() <= TOL[prec]
    if prec in TOL_MEDIAN:
        assert np.median(err) <= TOL_MEDIAN[prec]
    assert np.all(np.isfinite(a))


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32c", "fp32dl"])
def test_accel_ragged_batch_with_field(prec):
    torch_dev()
    b = _ragged_batch()
    sim = make_sim(b, prec)
    a = sim.accel().cpu().numpy()
    ref, scale = oracle_reference(b)
    err = rel_errors(a, ref, scale)
    print("\n[ragged %s] %s" % (prec, stats(err)), flush=True)
    if prec in TOL:
        assert err.max() <= TOL[prec]
    assert np.median(err) <= TOL_MEDIAN[prec]
    # the single-particle cluster without field feels exactly nothing
    sizes = np.diff(b.offsets)
    for c in np.nonzero(sizes == 1)[0]:
        if not b.field[c]:
            assert np.all(a[b.offsets[c]] == 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32dl"])
@pytest.mark.parametrize("shape", ["box300", "plummer6000"])
def test_zero_softening_masks_self_term(prec, shape):
    """eps = 0: the j = i term is excluded explicitly (potential too); the 6000-particle cluster is
    split into j-ranges and, in the local mode, has far tiles, so every masked loop runs."""
    torch_dev()
    p, v, m = inputs.uniform_box(300, 9) if shape == "box300" else inputs.plummer(6000, 31)
    b = inputs.single(p, v, m, 0.0)
    sim = make_sim(b, prec)
    a = sim.accel(pot=True).cpu().numpy()
    pot = sim.pot.cpu().numpy()
    ref, scale, rpot = oracle_reference(b, want_pot=True)
    err = rel_errors(a, ref, scale)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(pot))
    assert err.max() <= TOL[prec]
    assert np.abs(pot - rpot).max() <= (1e-13 if prec == "fp64" else 2e-6) * np.abs(rpot).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32dl"])
def test_potential(prec):
    torch_dev()
    b = _ragged_batch(seed=3)
    sim = make_sim(b, prec)
    sim.accel(pot=True)
    pot = sim.pot.cpu().numpy()
    _, _, rpot = oracle_reference(b, want_pot=True)
    rel = np.abs(pot - rpot) / np.maximum(np.abs(rpot), 1e-300)
    print("\n[pot %s] max rel %.3e" % (prec, rel.max()), flush=True)
    sizes = np.diff(b.offsets)
    ok = np.repeat(sizes > 1, sizes)
    assert rel[ok].max() <= (1e-13 if prec == "fp64" else 1e-6)
    assert np.all(pot[~ok] == 0)


def test_energy_fp64_matches_oracle():
    torch_dev()
    b = _ragged_batch(seed=5)
    sim = make_sim(b, "fp64")
    out = sim.energy().cpu().numpy()
    for c in range(b.B):
        s, e = b.offsets[c], b.offsets[c + 1]
        ref = oracle.energy(b.pos[s:e], b.vel[s:e], b.mass[s:e], b.G, b.eps[c], bool(b.field[c]), b.galaxy)
        scale = np.abs(ref[:4]).max()
        assert np.abs(out[c, :4] - ref[:4]).max() <= 1e-13 * scale + 1e-300
        assert np.abs(out[c, 4:14] - ref[4:14]).max() <= 1e-13 * (np.abs(ref[4:14]).max() + 1e-300)
        # internal force sum: zero up to rounding on both sides, its scale sum m |a_int| to 1e-13
        assert abs(out[c, 18] - ref[18]) <= 1e-13 * ref[18] + 1e-300
        assert np.abs(out[c, 14:18]).max() <= 1e-14 * ref[18] + 1e-300
        assert out[c, 19] == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32dl", "fp32c"])
def test_energy_internal_force_sum(prec):
    """sum m a_int = 0 (antisymmetry of the Eq. 2 pair forces): |F| / sum m |a_int| is at the
    rounding level of the mode's pair arithmetic, and sum m |a_int| matches the oracle's."""
    torch_dev()
    b = _ragged_batch(seed=11, sizes=(2, 255, 700, 3000, 9000))
    sim = make_sim(b, prec)
    out = sim.energy().cpu().numpy()
    tol = 1e-13 if prec == "fp64" else 1e-6
    for c in range(b.B):
        s, e = b.offsets[c], b.offsets[c + 1]
        ref = oracle.energy(b.pos[s:e], b.vel[s:e], b.mass[s:e], b.G, b.eps[c], bool(b.field[c]), b.galaxy)
        print("\n[force sum %s N=%d] |F|/sum m|a| gpu %.2e oracle %.2e" % (
            prec, e - s, out[c, 17] / out[c, 18], ref[17] / ref[18]), flush=True)
        assert out[c, 17] <= tol * out[c, 18]
        assert abs(out[c, 17] - np.linalg.norm(out[c, 14:17])) <= 1e-15 * out[c, 17] + 1e-300
        assert abs(out[c, 18] - ref[18]) <= tol * ref[18]


def test_energy_flags_nonfinite():
    torch_dev()
    p, v, m = inputs.plummer(300, 2)
    v[17, 1] = np.inf
    b = inputs.concat([inputs.single(p, v, m, 1e-3), inputs.single(*inputs.plummer(100, 3), 1e-3)])
    sim = make_sim(b, "fp64")
    out = sim.energy().cpu().numpy()
    assert out[0, 19] == 1.0 and out[1, 19] == 0.0


def test_leapfrog_trajectory_c1_fp64():
    """Plummer N=1024, eps=1e-3, 100 KDK steps of dt=1/1024 in FP64: positions agree with the
    oracle to 1e-10 relative, and the relative energy error matches the oracle's."""
    torch_dev()
    b = inputs.c1()
    sim = make_sim(b, "fp64")
    e0 = oracle.energy(b.pos, b.vel, b.mass, 1.0, 1e-3)[3]
    sim.accel()
    sim.step("leapfrog", 1.0 / 1024, 100)
    pos = sim.pos.cpu().numpy()
    vel = sim.vel.cpu().numpy()
    acc0 = oracle.total_accel(b.pos, b.mass, 1.0, 1e-3)
    rp, rv, ra = oracle.step(b.pos, b.vel, b.mass, acc0, 1.0 / 1024, 100, "leapfrog", 1.0, 1e-3)
    rel = np.abs(pos - rp).max() / np.abs(rp).max()
    print("\n[C1 trajectory] max rel pos diff %.3e" % rel, flush=True)
    assert rel <= 1e-10
    de_gpu = abs(oracle.energy(pos, vel, b.mass, 1.0, 1e-3)[3] - e0) / abs(e0)
    de_ref = abs(oracle.energy(rp, rv, b.mass, 1.0, 1e-3)[3] - e0) / abs(e0)
    print("[C1 energy] |dE/E0| gpu %.3e oracle %.3e" % (de_gpu, de_ref), flush=True)
    assert abs(de_gpu - de_ref) <= 1e-3 * de_ref + 1e-13
    a = sim.acc.cpu().numpy()
    ref, scale = oracle_reference(inputs.single(pos, vel, b.mass, 1e-3))
    assert rel_errors(a, ref, scale).max() <= TOL["fp64"]


def test_sym6_trajectory_with_field_fp64():
    torch_dev()
    b = _ragged_batch(seed=11, sizes=(130, 300), field_every=1, eps=1e-2)
    sim = make_sim(b, "fp64")
    sim.accel()
    dt = 1.0 / 256
    sim.step("sym6", dt, 6)
    pos = sim.pos.cpu().numpy()
    for c in range(b.B):
        s, e = b.offsets[c], b.offsets[c + 1]
        a0 = oracle.total_accel(b.pos[s:e], b.mass[s:e], 1.0, b.eps[c], True)
        rp, rv, _ = oracle.step(b.pos[s:e], b.vel[s:e], b.mass[s:e], a0, dt, 6, "sym6", 1.0, b.eps[c], True)
        assert np.abs(pos[s:e] - rp).max() <= 1e-10 * np.abs(rp).max()


def test_substep_per_cluster_coefficients():
    torch_dev()
    b = _ragged_batch(seed=13, sizes=(64, 200, 333))
    sim = make_sim(b, "fp64")
    sim.accel()
    kp = np.array([0.01, -0.003, 0.0])
    dr = np.array([0.02, 0.005, 0.01])
    kq = np.array([0.0, 0.004, 0.01])
    sim.substep(kp, dr, kq)
    pos = sim.pos.cpu().numpy()
    vel = sim.vel.cpu().numpy()
    for c in range(b.B):
        s, e = b.offsets[c], b.offsets[c + 1]
        a0 = oracle.total_accel(b.pos[s:e], b.mass[s:e], 1.0, b.eps[c], bool(b.field[c]))
        v = b.vel[s:e] + kp[c] * a0
        x = b.pos[s:e] + dr[c] * v
        a1 = oracle.total_accel(x, b.mass[s:e], 1.0, b.eps[c], bool(b.field[c]))
        v = v + kq[c] * a1
        assert np.abs(pos[s:e] - x).max() <= 1e-14 * np.abs(x).max()
        assert np.abs(vel[s:e] - v).max() <= 1e-12 * np.abs(v).max()


def test_deterministic_and_alone_equals_in_batch():
    torch_dev()
    b = _ragged_batch(seed=17)
    sim = make_sim(b, "fp32ds")
    a1 = sim.accel().cpu().numpy().copy()
    a2 = sim.accel().cpu().numpy()
    assert np.array_equal(a1, a2)
    for c in (4, 7):
        s, e = b.offsets[c], b.offsets[c + 1]
        alone = inputs.single(b.pos[s:e], b.vel[s:e], b.mass[s:e], b.eps[c], bool(b.field[c]))
        sa = make_sim(alone, "fp32ds")
        assert np.array_equal(sa.accel().cpu().numpy(), a1[s:e])


def test_full_size_c3_sampled_rows():
    """N = 262144 (the benchmark's workload) in the benchmark's launch shape: sampled rows checked
    one by one against the oracle, plus momentum conservation over all particles."""
    torch_dev()
    b = inputs.c3()
    for prec in ("fp32ds", "fp32c", "fp64", "fp32dl"):
        sim = make_sim(b, prec)
        a = sim.accel().cpu().numpy()
        rows = [(0, 64), (131072 - 32, 131072 + 32), (262144 - 64, 262144)]
        errs = []
        for r0, r1 in rows:
            ref, absa = oracle.accel(b.pos, b.mass, 1.0, 1e-4, rows=(r0, r1), want_abs=True)
            errs.append(rel_errors(a[r0:r1], ref, absa))
        err = np.concatenate(errs)
        print("\n[C3 %s sampled] %s" % (prec, stats(err)), flush=True)
        if prec in TOL:
            assert err.max() <= TOL[prec]
        assert np.median(err) <= TOL_MEDIAN[prec]
        mom = np.abs((b.mass[:, None] * a).sum(0)).max() / (b.mass[:, None] * np.abs(a)).sum()
        assert mom < (1e-12 if prec == "fp64" else 1e-6)
        sim.close()


def test_full_size_c2_sampled_rows_with_field():
    """N = 65536 with Salpeter masses, eps = 1e-4 and the galaxy field (the sym6 workload): sampled
    rows against the oracle (internal + field), with per-row scales."""
    torch_dev()
    b = inputs.c2()
    rows = [(0, 64), (32768 - 32, 32768 + 32), (65536 - 64, 65536)]
    for prec in ("fp64", "fp32ds", "fp32c", "fp32dl"):
        sim = make_sim(b, prec)
        a = sim.accel().cpu().numpy()
        errs = []
        for r0, r1 in rows:
            ref, absa = oracle.accel(b.pos, b.mass, 1.0, 1e-4, rows=(r0, r1), want_abs=True)
            ae, _ = oracle.ext_field(b.pos[r0:r1], 1.0, b.galaxy)
            errs.append(rel_errors(a[r0:r1], ref + ae, absa + np.linalg.norm(ae, axis=1)))
        err = np.concatenate(errs)
        print("\n[C2 %s sampled] %s" % (prec, stats(err)), flush=True)
        if prec in TOL:
            assert err.max() <= TOL[prec]
        assert np.median(err) <= TOL_MEDIAN[prec]
        sim.close()


def test_full_size_c4_sampled_clusters():
    """The 512-cluster ensemble in one launch: the smallest, the largest and clusters of each split
    class checked whole against the oracle."""
    torch_dev()
    b = inputs.c4()
    sizes = np.diff(b.offsets)
    order = np.argsort(sizes)
    pick = sorted(set([int(order[0]), int(order[-1])] + [int(order[np.searchsorted(sizes[order], n)])
                                                         for n in (1024, 2048, 4096, 9000)]))
    for prec in ("fp32ds", "fp64", "fp32dl"):
        sim = make_sim(b, prec)
        a = sim.accel().cpu().numpy()
        errs = []
        for c in pick:
            s, e = b.offsets[c], b.offsets[c + 1]
            ref, _, absa = oracle.accel(b.pos[s:e], b.mass[s:e], 1.0, 1e-3, want_pot=True, want_abs=True)
            errs.append(rel_errors(a[s:e], ref, absa))
        err = np.concatenate(errs)
        print("\n[C4 %s clusters %s] %s" % (prec, [int(sizes[c]) for c in pick], stats(err)), flush=True)
        assert err.max() <= TOL[prec]
        assert np.median(err) <= TOL_MEDIAN[prec]
        sim.close()


@pytest.mark.parametrize("prec", ["fp32ds", "fp32c"])
@pytest.mark.parametrize("tile", [(2, 4, 256, 4, 1), (1, 4, 256, 8, 1), (2, 2, 256, 4, 1), (2, 4, 128, 8, 1),
                                  (1, 1, 128, 2, 0), (1, 2, 256, 8, 0)])
def test_launch_shapes_agree(prec, tile):
    """Every launch shape (including the rsq-phased loop) meets the same accuracy bound; shapes with
    the same tile and waves per group give bitwise the same result."""
    torch_dev()
    from paper_1003_3896_amd import nbody
    p, v, m = inputs.plummer(3000, 4321)
    b = inputs.single(p, v, m, 1e-3)
    sim = make_sim(b, prec)
    for ncl in range(nbody.N_CLASSES):
        nbody.nbody_set_tile(sim.ctx, prec, ncl, *tile)
    a = sim.accel().cpu().numpy().copy()
    ref, scale = oracle_reference(b)
    err = rel_errors(a, ref, scale)
    if prec in TOL:
        assert err.max() <= TOL[prec]
    assert np.median(err) <= TOL_MEDIAN[prec]
    if tile[4] == 1:  # the phased loop does the same arithmetic per term as the plain one
        for ncl in range(nbody.N_CLASSES):
            nbody.nbody_set_tile(sim.ctx, prec, ncl, *tile[:4], 0)
        assert np.array_equal(sim.accel().cpu().numpy(), a)


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32c", "fp32dl"])
def test_equal_and_nearly_equal_masses(prec):
    """Clusters whose masses are all equal take the path that scales the mass-free sums by the
    common mass once; one different mass anywhere (first particle, last chunk, a split cluster)
    must take the weighted path.  Both match the oracle, potential included."""
    torch_dev()
    cl = []
    for c, (n, odd) in enumerate(((700, None), (1300, -1), (1300, 0), (3000, None), (3000, 2999), (5, None))):
        p, v, m = inputs.plummer(n, 4400 + c)
        m = m.copy()
        if odd is not None:
            m[odd] *= 1.5
        cl.append(inputs.single(p, v, m, 1e-3 if c != 5 else 0.0, False))
    b = inputs.concat(cl)
    sim = make_sim(b, prec)
    a = sim.accel(pot=True).cpu().numpy()
    pot = sim.pot.cpu().numpy()
    ref, scale, rpot = oracle_reference(b, want_pot=True)
    err = rel_errors(a, ref, scale)
    print("\n[masses %s] %s" % (prec, stats(err)), flush=True)
    if prec in TOL:
        assert err.max() <= TOL[prec]
    assert np.median(err) <= TOL_MEDIAN[prec]
    ptol = {"fp64": 1e-13, "fp32ds": 2e-6, "fp32c": 1e-5, "fp32dl": 2e-6}[prec]
    for c in range(b.B):
        s, e = b.offsets[c], b.offsets[c + 1]
        assert np.abs(pot[s:e] - rpot[s:e]).max() <= ptol * np.abs(rpot[s:e]).max(), c


@pytest.mark.parametrize("tile", [(2, 4, 256, 4, 0), (2, 2, 256, 8, 0), (1, 4, 128, 8, 0), (2, 4, 128, 4, 0),
                                  (1, 4, 256, 8, 0), (1, 2, 256, 8, 0), (1, 2, 128, 4, 0)])
def test_local_mode_shapes_and_order(tile):
    """The Hilbert-sorted local mode returns every particle's result at its own index and meets the
    double-single bound in every compiled shape on a cluster large enough to have far tiles;
    repeated evaluations are bitwise identical."""
    torch_dev()
    from paper_1003_3896_amd import nbody
    p, v, m = inputs.plummer(20000, 4711)
    b = inputs.single(p, v, m, 1e-3)
    sim = make_sim(b, "fp32dl")
    for ncl in range(nbody.N_CLASSES):
        nbody.nbody_set_tile(sim.ctx, "fp32dl", ncl, *tile)
    a = sim.accel().cpu().numpy().copy()
    assert np.array_equal(sim.accel().cpu().numpy(), a)
    ref, scale = oracle_reference(b)
    err = rel_errors(a, ref, scale)
    print("\n[fp32dl %s] %s" % (tile, stats(err)), flush=True)
    assert err.max() <= TOL["fp32dl"]
    assert np.median(err) <= TOL_MEDIAN["fp32dl"]
    # blocks per CU (the grid) change nothing
    for ncl in range(nbody.N_CLASSES):
        nbody.nbody_set_tile(sim.ctx, "fp32dl", ncl, *tile[:3], 2, 0)
    assert np.array_equal(sim.accel().cpu().numpy(), a)


@pytest.mark.parametrize("masses", ["equal", "salpeter"])
@pytest.mark.parametrize("tile", [(1, 4, 256, 8, 0), (2, 4, 128, 4, 0)])
def test_local_mode_unsoftened(tile, masses):
    """eps = 0 (the self term masked), with equal masses (where most far tiles take the expanded
    form of r^2 with one particle per lane) and with Salpeter masses (the direct far-tile loop with
    a mass per source), and a trailing one-particle item (zero box, so every full tile of it is
    far): the accelerations meet the double-single bound and the potentials match the oracle."""
    torch_dev()
    from paper_1003_3896_amd import nbody
    p, v, m = inputs.plummer(16385, 4712, salpeter=masses == "salpeter")
    b = inputs.single(p, v, m, 0.0)
    sim = make_sim(b, "fp32dl")
    for ncl in range(nbody.N_CLASSES):
        nbody.nbody_set_tile(sim.ctx, "fp32dl", ncl, *tile)
    a = sim.accel(pot=True).cpu().numpy()
    pot = sim.pot.cpu().numpy()
    assert np.isfinite(a).all() and np.isfinite(pot).all()
    ref, scale, rpot = oracle_reference(b, want_pot=True)
    err = rel_errors(a, ref, scale)
    print("\n[fp32dl eps=0 %s %s] %s" % (tile, masses, stats(err)), flush=True)
    assert err.max() <= TOL["fp32dl"]
    assert np.median(err) <= TOL_MEDIAN["fp32dl"]
    assert np.abs(pot - rpot).max() <= 2e-6 * np.abs(rpot).max()


def test_local_mode_coincident_particles():
    """Items whose particles all sit at one point (a zero box: every full tile is far and expanded,
    the frame centred on that point) and sources coincident with them, softened: the local mode
    meets the double-single bound against the oracle."""
    torch_dev()
    p, v, m = inputs.plummer(3000, 4713)
    p = p.copy()
    p[:200] = p[0]            # 200 particles at one point (three whole items and part of a fourth)
    p[1500:1520] = p[0]       # and some sources far away in the order at the same point
    b = inputs.single(p, v, m, 1e-3)
    sim = make_sim(b, "fp32dl")
    a = sim.accel().cpu().numpy()
    assert np.isfinite(a).all()
    ref, scale = oracle_reference(b)
    err = rel_errors(a, ref, scale)
    print("\n[fp32dl coincident] %s" % stats(err), flush=True)
    assert err.max() <= TOL["fp32dl"]


def test_local_mode_alone_equals_in_batch():
    """With one launch shape for every size class, a cluster's local-mode result (sort, item
    boxes, near/far choices) is bitwise the same alone and in a ragged batch."""
    torch_dev()
    from paper_1003_3896_amd import nbody
    b = _ragged_batch(seed=23, sizes=(5, 300, 2500, 9000, 17), field_every=2)

    def run(batch):
        sim = make_sim(batch, "fp32dl")
        for ncl in range(nbody.N_CLASSES):
            nbody.nbody_set_tile(sim.ctx, "fp32dl", ncl, 2, 4, 256, 4, 0)
        return sim.accel().cpu().numpy().copy()

    a1 = run(b)
    ref, scale = oracle_reference(b)
    assert rel_errors(a1, ref, scale).max() <= TOL["fp32dl"]
    for c in (1, 2, 3):
        s, e = b.offsets[c], b.offsets[c + 1]
        alone = inputs.single(b.pos[s:e], b.vel[s:e], b.mass[s:e], b.eps[c], bool(b.field[c]))
        assert np.array_equal(run(alone), a1[s:e]), c


@pytest.mark.parametrize("prec", ["fp64", "fp32ds", "fp32dl"])
def test_black_hole_field(prec):
    """Sect. 6.2's central point mass in the field: a cluster passing close to it (the stiff case)
    matches the oracle, internal and external terms together; in FP64 also along 10 sym6 steps."""
    torch_dev()
    b = inputs.paper_black_hole(50.0, n=2048)
    b.pos = b.pos - np.array([9.95, 0.0, 0.0])  # barycentre 0.05 from the black hole
    sim = make_sim(b, prec)
    a = sim.accel().cpu().numpy()
    ref, scale = oracle_reference(b)
    err = rel_errors(a, ref, scale)
    print("\n[black hole %s] %s" % (prec, stats(err)), flush=True)
    assert err.max() <= TOL[prec]
    if prec == "fp64":
        dt = 1e-4
        a0 = oracle.total_accel(b.pos, b.mass, 1.0, b.eps[0], True, b.galaxy)
        rp, rv, _ = oracle.step(b.pos, b.vel, b.mass, a0, dt, 10, "sym6", 1.0, b.eps[0], True, b.galaxy)
        sim.step("sym6", dt, 10)
        pos = sim.pos.cpu().numpy()
        assert np.abs(pos - rp).max() <= 1e-10 * np.abs(rp).max()
        e_gpu = sim.energy(prec="fp64")[0].cpu().numpy()
        e_ref = oracle.energy(rp, rv, b.mass, 1.0, b.eps[0], True, b.galaxy)
        assert abs(e_gpu[3] - e_ref[3]) <= 1e-11 * abs(e_ref[3])
