"""GPU parity for the indirect system and the fields off the surface.

  indirect assembly  msv_assemble with formulation 1 (eq. dualmullrep) on the
                     ORACLE table vs oracle.assemble(formulation="indirect")
                     on the same table, with the per-row bound of the direct
                     system's assembly test (1e-12 of the row, or 16 times the
                     oracle's own change under one-ulp table noise).
  far field, fields  msv_far_field / msv_fields on the GPU's currents vs
                     oracle.farfield / oracle.fields on the same currents:
                     both evaluate the same surface quadrature (same azimuth
                     count), so they agree to rounding: 1e-12 relative.
  extinction         the current-loop test of Section 6 end to end on the GPU
                     (tabulate, assemble, factor, solve in both precisions,
                     interior field by eq. interior_dual): E_error below the
                     2.32e-9 that Table 1 prints for k0 = 1, k1 = 2, the
                     exterior field below 5e-9 of the loop field, and the
                     currents equal to the oracle's to max(1e-10, 4 sens)
                     (L2-weighted), sens being the oracle's own change under
                     1e-14 kernel noise.
  starfish, droplet, the same test at the sizes of the first rows of Tables 2,
  cylinder           3 and 4 (a body reaching toward the loop; a conical
                     point on the axis; edges with corner panels near 1e-5),
                     E_error below the printed values; the starfish's and the
                     droplet's currents against the oracle's, the cylinder's
                     interior fields against stored oracle fields.
  extinction theorem for the direct system on the sphere: the exterior
                     representation evaluated inside is -E_inc (3e-9, the
                     oracle's own floor on this body).
"""
import json
import os

import numpy as np
import pytest

from gpu_cases import RULES, oracle_setup, oracle_table
from oracle import assemble as oasm
from oracle import farfield, fields
from oracle import solve as osolve
from oracle.modal import KernelParams
from workloads import geometry, incident

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1810_07067_amd as msv  # noqa: E402

LOOP = dict(center=[0.4, 0.5, 5.0], radius=0.42)


def _plan(curve, k0, eps1, mu1, M, L, precision=0, formulation=0):
    print(f"[case] {curve.name} N={curve.n} k0={k0} eps1={eps1} mu1={mu1} M={M} L={L} prec={precision} "
          f"formulation={formulation}", flush=True)
    return msv.plan_from_curve(curve, RULES, k0, eps1, mu1, m_max=M, fft_len=L, precision=precision,
                               formulation=formulation)


def _rel(got, ref, floor=0.0):
    """max |got - ref| over max |ref|, the latter at least `floor` (for a
    reference that vanishes, the size of the fields it is measured against)."""
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), floor))


def e_error(E, H, Er, Hr):
    num = np.linalg.norm(E - Er) ** 2 + np.linalg.norm(H - Hr) ** 2
    return float(np.sqrt(num / (np.linalg.norm(Er) ** 2 + np.linalg.norm(Hr) ** 2)))


def torus_points(rng, P, frac=0.5):
    rho = frac * np.sqrt(rng.uniform(0, 1, P))
    ph = rng.uniform(0, 2 * np.pi, P)
    th = rng.uniform(0, 2 * np.pi, P)
    rr = 2 + rho * np.cos(ph)
    zz = 0.5 * rho * np.sin(ph)
    return np.stack([rr * np.cos(th), rr * np.sin(th), zz], axis=1)


@pytest.fixture(scope="module", params=[(4.0, 1.0), (2.0, 2.0)], ids=["dielectric", "magnetic"])
def torus(request):
    """Table 1, first row: the torus of Example 1, k0 = 1, k1 = 2, N_f = 13."""
    eps1, mu1 = request.param
    curve, k0, M, L = geometry.torus(8), 1.0, 13, 128
    sup, kp = oracle_setup(curve, k0, eps1, M, L, mu1=mu1)
    tab = oracle_table(curve, sup, kp)
    w = geometry.gl_weights(curve)
    args = (k0, kp.k1, k0, 1.0, 1.0, eps1, mu1, w)
    mats = np.array([oasm.assemble_mode(curve, sup, tab, m, *args, formulation="indirect") for m in range(M + 1)])
    rng = np.random.default_rng(11)
    tabp = tab * (1.0 + 2.0 ** -53 * rng.uniform(-1.0, 1.0, tab.shape))
    matsp = np.array([oasm.assemble_mode(curve, sup, tabp, m, *args, formulation="indirect")
                      for m in range(M + 1)])
    rhs = incident.loop_rhs_modes(curve, LOOP["center"], LOOP["radius"], kp.k1, k0, mu1, -M, M)
    x = osolve.solve_modes(list(mats), w, rhs, -M, M)
    # the oracle's own change of the currents when every kernel moves by 1e-14
    # (the accuracy both implementations reach): the GPU's currents are held
    # to max(1e-10, 4 x that), as in the direct system's end-to-end test
    tabk = tab * (1.0 + 1e-14 * np.random.default_rng(12).uniform(-1.0, 1.0, tab.shape))
    matsk = [oasm.assemble_mode(curve, sup, tabk, m, *args, formulation="indirect") for m in range(M + 1)]
    xk = osolve.solve_modes(matsk, w, rhs, -M, M)
    sw = np.sqrt(np.repeat(w, 4))
    sens_x = np.linalg.norm(sw * (x - xk)) / np.linalg.norm(sw * x)
    return dict(curve=curve, k0=k0, eps1=eps1, mu1=mu1, M=M, L=L, k1=kp.k1, tab=tab, mats=mats, matsp=matsp,
                w=w, rhs=rhs, x=x, sens_x=sens_x)


def test_indirect_assembly_parity(torus):
    c = torus
    plan = _plan(c["curve"], c["k0"], c["eps1"], c["mu1"], c["M"], c["L"], formulation=1)
    A = plan.assemble(torch.from_numpy(c["tab"]).cuda(), 0, c["M"]).cpu().numpy()
    ref = c["mats"]
    diff = np.max(np.abs(A - ref), axis=(0, 2))
    rowmax = np.max(np.abs(ref), axis=(0, 2))
    sens = np.max(np.abs(c["matsp"] - ref), axis=(0, 2))
    bound = np.maximum(1e-12 * rowmax, 16.0 * sens)
    print(f"[indirect assemble] max row err/rowmax {np.max(diff / rowmax):.3e}", flush=True)
    assert np.all(diff <= bound), np.max(diff / bound)


@pytest.mark.parametrize("precision", [0, 1])
def test_extinction_end_to_end(torus, precision):
    c = torus
    curve, M = c["curve"], c["M"]
    plan = _plan(curve, c["k0"], c["eps1"], c["mu1"], M, c["L"], precision=precision, formulation=1)
    kern = plan.tabulate()
    A = plan.assemble(kern, 0, M)
    plan.factor(A, 0, M)
    x = plan.solve(-M, M, torch.from_numpy(c["rhs"]).cuda())
    xh = x.cpu().numpy()
    sw = np.sqrt(np.repeat(c["w"], 4))
    cur = np.linalg.norm(sw * (xh - c["x"])) / np.linalg.norm(sw * c["x"])
    pts = torus_points(np.random.default_rng(3), 6)
    E, H = plan.fields(-M, M, x, pts, "interior")
    El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], c["k1"], c["k0"], c["mu1"])
    err = e_error(E[0].cpu().numpy(), H[0].cpu().numpy(), El(pts), Hl(pts))
    out = np.array([[0.0, 0.0, 0.3], [4.0, 0.5, 0.2], [-3.5, -1.0, 1.2], [0.5, 0.2, -1.5]])
    Ee, He = plan.fields(-M, M, x, out, "exterior")
    scale = np.sqrt(np.linalg.norm(El(pts)) ** 2 + np.linalg.norm(Hl(pts)) ** 2)
    ext = np.sqrt(np.linalg.norm(Ee.cpu().numpy()) ** 2 + np.linalg.norm(He.cpu().numpy()) ** 2) / scale
    print(f"[extinction] eps1={c['eps1']} mu1={c['mu1']} prec {precision}: E_error {err:.3e}, exterior {ext:.3e}, "
          f"currents vs oracle {cur:.3e} (oracle sensitivity {c['sens_x']:.3e})", flush=True)
    assert cur < max(1e-10, 4.0 * c["sens_x"]), cur
    assert err < 2.32e-9, err
    assert ext < 5e-9, ext
    # the GPU's field evaluation against the oracle's on the same currents
    Eo, Ho = fields.fields(curve, c["w"], xh[:, 0], -M, pts, c["k0"], c["k1"], c["k0"], 1.0, 1.0, c["eps1"],
                           c["mu1"], "interior", "indirect")
    assert _rel(E[0].cpu().numpy(), Eo) < 1e-12 and _rel(H[0].cpu().numpy(), Ho) < 1e-12


def test_extinction_at_the_paper_size():
    """Table 1's first row at its own size (64 points): the GPU path end to end
    with the field evaluation on 4 sub-panels per panel, below the printed
    E_error 2.32e-9."""
    curve, k0, eps1, M, L = geometry.torus(4), 1.0, 4.0, 13, 128
    k1 = k0 * np.sqrt(eps1)
    plan = _plan(curve, k0, eps1, 1.0, M, L, precision=1, formulation=1)
    A = plan.assemble(plan.tabulate(), 0, M)
    plan.factor(A, 0, M)
    rhs = incident.loop_rhs_modes(curve, LOOP["center"], LOOP["radius"], k1, k0, 1.0, -M, M)
    x = plan.solve(-M, M, torch.from_numpy(rhs).cuda())
    pts = torus_points(np.random.default_rng(3), 6)
    El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], k1, k0, 1.0)
    E, H = plan.fields(-M, M, x, pts, "interior", upsample=4)
    err = e_error(E[0].cpu().numpy(), H[0].cpu().numpy(), El(pts), Hl(pts))
    print(f"[extinction] 64 points, upsample 4: E_error {err:.3e}", flush=True)
    assert err < 2.32e-9, err


def _loop_solve(curve, k0, k1, M, L, precision):
    """Tabulate, assemble, factor and solve the indirect system for the loop
    data; complex64 factors whose refinement does not converge fall back to
    complex128, as the extinction form does."""
    eps1 = (k1 / k0) ** 2
    rhs = torch.from_numpy(incident.loop_rhs_modes(curve, LOOP["center"], LOOP["radius"], k1, k0, 1.0,
                                                   -M, M)).cuda()
    for prec in (precision, 0):
        plan = _plan(curve, k0, eps1, 1.0, M, L, precision=prec, formulation=1)
        A = plan.assemble(plan.tabulate(), 0, M)
        plan.factor(A, 0, M)
        try:
            return plan, plan.solve(-M, M, rhs), rhs
        except msv.MsvError as exc:
            if exc.status != msv.MSV_ENOCONV or prec == 0:
                raise
            print("[extinction] refinement did not converge: complex128 LU", flush=True)
            plan.close()


def droplet_points(rng, P):
    t = rng.uniform(0.6, 0.9, P)
    sc = rng.uniform(0.0, 0.5, P)
    th = rng.uniform(0, 2 * np.pi, P)
    rr = sc * np.sin(np.pi * t) * np.cos(0.5 * np.pi * (t - 1.5))
    zz = np.sin(np.pi * t) * np.sin(0.5 * np.pi * (t - 1.5)) + 0.5
    return np.stack([rr * np.cos(th), rr * np.sin(th), zz], axis=1)


def test_extinction_droplet():
    """Table 3's first row: k0 = 5, k1 = 2, N_f = 7, 224 points (14 panels,
    five dyadic levels at the tip); printed E_error 2.71e-10."""
    curve, k0, k1, M, L = geometry.droplet(14), 5.0, 2.0, 7, 64
    sup, kp = oracle_setup(curve, k0, (k1 / k0) ** 2, M, L)
    while not kp.valid:
        L *= 2
        sup, kp = oracle_setup(curve, k0, (k1 / k0) ** 2, M, L)
    tab = oracle_table(curve, sup, kp)
    w = geometry.gl_weights(curve)
    args = (k0, kp.k1, k0, 1.0, 1.0, (k1 / k0) ** 2, 1.0, w)
    mats = [oasm.assemble_mode(curve, sup, tab, m, *args, formulation="indirect") for m in range(M + 1)]
    plan, x, rhs = _loop_solve(curve, k0, k1, M, L, 1)
    xo = osolve.solve_modes(mats, w, rhs.cpu().numpy(), -M, M)
    sw = np.sqrt(np.repeat(w, 4))
    cur = np.linalg.norm(sw * (x.cpu().numpy() - xo)) / np.linalg.norm(sw * xo)
    pts = droplet_points(np.random.default_rng(3), 6)
    E, H = plan.fields(-M, M, x, pts, "interior", upsample=4)
    El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], k1, k0, 1.0)
    err = e_error(E[0].cpu().numpy(), H[0].cpu().numpy(), El(pts), Hl(pts))
    print(f"[extinction] droplet 224 points: E_error {err:.3e}, currents vs oracle {cur:.3e}", flush=True)
    assert cur < 1e-10, cur
    assert err < 2.71e-10, err


def test_extinction_starfish():
    """Table 2's first row: the rotated starfish of Example 2, k0 = 5, k1 = 2,
    N_f = 10, 224 points (14 equal panels in t); printed E_error 1.24e-9.  The
    currents against the oracle's on the same system."""
    curve, k0, k1, M, L = geometry.starfish(14), 5.0, 2.0, 10, 64
    sup, kp = oracle_setup(curve, k0, (k1 / k0) ** 2, M, L)
    while not kp.valid:
        L *= 2
        sup, kp = oracle_setup(curve, k0, (k1 / k0) ** 2, M, L)
    tab = oracle_table(curve, sup, kp)
    w = geometry.gl_weights(curve)
    args = (k0, kp.k1, k0, 1.0, 1.0, (k1 / k0) ** 2, 1.0, w)
    mats = [oasm.assemble_mode(curve, sup, tab, m, *args, formulation="indirect") for m in range(M + 1)]
    plan, x, rhs = _loop_solve(curve, k0, k1, M, L, 1)
    xo = osolve.solve_modes(mats, w, rhs.cpu().numpy(), -M, M)
    sw = np.sqrt(np.repeat(w, 4))
    cur = np.linalg.norm(sw * (x.cpu().numpy() - xo)) / np.linalg.norm(sw * xo)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((6, 3))
    pts = v / np.linalg.norm(v, axis=1)[:, None] * rng.uniform(0, 0.75, (6, 1))  # inside the ball of radius 1.5
    E, H = plan.fields(-M, M, x, pts, "interior", upsample=4)
    El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], k1, k0, 1.0)
    err = e_error(E[0].cpu().numpy(), H[0].cpu().numpy(), El(pts), Hl(pts))
    print(f"[extinction] starfish 224 points: E_error {err:.3e}, currents vs oracle {cur:.3e}", flush=True)
    assert cur < 1e-10, cur
    assert err < 1.24e-9, err


def test_extinction_cylinder():
    """Table 4's first row: k0 = 2, k1 = 1, N_f = 9, about 1312 points (81
    panels: 26 base panels, the four corner panels refined 14 levels down to
    about 1e-5); printed E_error 4.11e-9.  The interior fields also against
    the oracle's (tests/golden/extinction_cylinder_row1.json, written by
    make_extinction_cylinder.py from oracle/ alone) to 1e-10 relative, the
    far-field bar, below the E_error itself."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "extinction_cylinder_row1.json")))
    curve, k0, k1, M, L = geometry.cylinder(14, 6.5), 2.0, 1.0, 9, 64
    while not KernelParams(k0, k1, M, L, float(curve.r.max())).valid:
        L *= 2
    assert (curve.n, L) == (int(gold["body"].split("N = ")[1]), gold["L"])
    plan, x, _ = _loop_solve(curve, k0, k1, M, L, 1)
    pts = np.array(gold["points"])
    E, H = plan.fields(-M, M, x, pts, "interior", upsample=4)
    E, H = E[0].cpu().numpy(), H[0].cpu().numpy()
    El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], k1, k0, 1.0)
    err = e_error(E, H, El(pts), Hl(pts))
    cplx = lambda a: np.array([complex(*v) for v in a]).reshape(-1, 3)
    Eo, Ho = cplx(gold["E"]), cplx(gold["H"])
    scale = max(np.abs(Eo).max(), np.abs(Ho).max())
    par = max(np.abs(E - Eo).max(), np.abs(H - Ho).max()) / scale
    print(f"[extinction] cylinder {curve.n} points: E_error {err:.3e} (oracle {gold['E_error']:.3e}), "
          f"fields vs oracle {par:.3e}", flush=True)
    assert err < 4.11e-9, err
    assert par < 1e-10, par


@pytest.fixture(scope="module")
def sphere():
    curve, k0, eps1, M, L = geometry.sphere(8), 1.0, 2.25, 16, 64
    plan = _plan(curve, k0, eps1, 1.0, M, L)
    kern = plan.tabulate()
    A = plan.assemble(kern, 0, M)
    plan.factor(A, 0, M)
    waves = [incident.tilted_direction(30.0), incident.random_directions(9, 1)[0]]
    rhs = incident.rhs_modes(curve, waves, k0, -M, M)
    x = plan.solve(-M, M, torch.from_numpy(rhs).cuda())
    return dict(curve=curve, k0=k0, eps1=eps1, M=M, plan=plan, x=x, xh=x.cpu().numpy(), waves=waves,
                w=geometry.gl_weights(curve), k1=k0 * np.sqrt(eps1))


def test_far_field_parity(sphere):
    s = sphere
    rng = np.random.default_rng(4)
    dirs = rng.standard_normal((37, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    got = s["plan"].far_field(-s["M"], s["M"], s["x"], dirs).cpu().numpy()
    for v in range(2):
        ref = farfield.far_field(s["curve"], s["w"], s["xh"][:, v], -s["M"], s["k0"], s["k0"], 1.0, dirs)
        err = _rel(got[v], ref)
        print(f"[far field] vector {v}: {err:.3e}", flush=True)
        assert err < 1e-12, err


def test_fields_parity_and_extinction_theorem(sphere):
    s = sphere
    M, curve = s["M"], s["curve"]
    inside = np.array([[0.1, 0.2, -0.1], [-0.3, 0.1, 0.35], [0.0, -0.4, 0.2]])
    outside = np.array([[2.0, 0.5, -0.3], [-1.0, -1.5, 1.2], [0.2, 0.1, -2.5], [0.0, 0.0, 1.6]])
    cases = [("exterior", inside, 1), ("exterior", outside, 1), ("interior", inside, 1), ("interior", outside, 1),
             ("interior", inside, 4), ("exterior", outside, 3), ("interior", inside, 2)]
    for region, pts, U in cases:
        E, H = s["plan"].fields(-M, M, s["x"], pts, region, upsample=U)
        E, H = E.cpu().numpy(), H.cpu().numpy()
        for v in range(2):
            Eo, Ho = fields.fields(curve, s["w"], s["xh"][:, v], -M, pts, s["k0"], s["k1"], s["k0"], 1.0, 1.0,
                                   s["eps1"], 1.0, region, upsample=U)
            # the interior representation vanishes outside (extinction theorem):
            # there the difference is measured against the unit incident field
            err = max(_rel(E[v], Eo, 1e-2), _rel(H[v], Ho, 1e-2))
            print(f"[fields] {region} ({len(pts)} points, upsample {U}) vector {v}: {err:.3e}", flush=True)
            assert err < 1e-12, err
        if region == "exterior" and pts is inside and U == 1:
            for v, (d, p) in enumerate(s["waves"]):
                Ei, Hi = incident.plane_wave(d, p, s["k0"])
                assert e_error(E[v], H[v], -Ei(pts), -Hi(pts)) < 3e-9
