"""GPU parity: the HIP library (through the C ABI) against the CPU oracle
on the same seeded inputs.

Tolerances: FP64 untruncated runs must reproduce the dense oracle to the
rounding level of the algebra (1e-10 relative, a few hundred FP64
operations deep per entry); truncated runs are compared with the CPU MPS
oracle running the same schedule, where both sides truncate at the same
tolerance, so the bound is a small multiple of that tolerance.
"""
import numpy as np
import pytest

import workloads as WL
from oracle.dense_lbm import DenseLBM
from oracle.mps_lbm import MPSLBM

pytestmark = pytest.mark.gpu


def lib():
    from paper_2512_07615_amd import mps_lbm as L
    L.load()
    return L


def _hip_stream():
    """A non-default stream from the HIP runtime the library itself uses
    (created through ctypes, so that no second runtime gets loaded)."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so.7")
    s = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(s)) == 0
    return s.value


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _case_with_flow(case, seed=3, amp=0.01):
    rho, u = WL.random_flow_state(case.n, seed, amp=amp)
    case.rho_init, case.u_init = rho, u
    return case


def test_init_roundtrip_fp64():
    L = lib()
    case = _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-14))
    print("case", case.name, flush=True)
    sim = L.Simulation(case, precision="fp64")
    got = sim.dense(L.POPS)
    ref = DenseLBM(case).f
    sim.close()
    assert rel(got, ref) < 1e-12


def test_one_step_channel8_fp64():
    L = lib()
    case = _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13))
    sim = L.Simulation(case, precision="fp64")
    sim.step(1)
    got = sim.dense(L.POPS)
    d = DenseLBM(case)
    d.step()
    obs = sim.observables()
    sim.close()
    print("rel", rel(got, d.f), "roundings", obs.roundings, "products", obs.products, flush=True)
    assert rel(got, d.f) < 1e-10


@pytest.mark.parametrize("which", ["porous16", "vascular16"])
def test_open_faces_untruncated_fp64(which):
    L = lib()
    if which == "porous16":
        case = WL.case_porous(n=4, chi=64, tol=1e-13)
    else:
        case = WL.case_vascular(n=4, chi=64, tol=1e-13)
    case = _case_with_flow(case)
    sim = L.Simulation(case, precision="fp64")
    d = DenseLBM(case)
    for _ in range(2):
        sim.step(1)
        d.step()
    got = sim.dense(L.POPS)
    sim.close()
    assert rel(got, d.f) < 1e-10


def test_channel16_chi16_fp64_vs_oracles():
    """The 16^3 body-force channel at chi = 16, tol 1e-10 (FP64)."""
    L = lib()
    case = WL.case_channel()
    sim = L.Simulation(case, precision="fp64")
    m = MPSLBM(case)
    d = DenseLBM(case)
    for _ in range(20):
        sim.step(1)
        m.step()
        d.step()
    got = sim.dense(L.POPS)
    obs = sim.observables()
    sim.close()
    assert rel(got, d.f) < 1e-9
    assert rel(got, m.dense_populations()) < 1e-9
    assert abs(obs.mass - m.mass()) / m.mass() < 1e-12


def test_one_step_channel8_fp32():
    L = lib()
    case = _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-7))
    sim = L.Simulation(case, precision="fp32")
    sim.step(1)
    got = sim.dense(L.POPS)
    d = DenseLBM(case)
    d.step()
    sim.close()
    assert rel(got, d.f) < 2e-5


@pytest.mark.parametrize("which", ["porous16", "vascular16"])
def test_open_faces_untruncated_fp32(which):
    """FP32 policy, untruncated (chi at full rank): the dense oracle is the
    reference; the bound is FP32 rounding accumulated over two steps (each
    value passes some tens of roundings of relative size ~1e-7)."""
    L = lib()
    if which == "porous16":
        case = WL.case_porous(n=4, chi=64, tol=1e-7)
    else:
        case = WL.case_vascular(n=4, chi=64, tol=1e-7)
    case = _case_with_flow(case)
    sim = L.Simulation(case, precision="fp32")
    d = DenseLBM(case)
    for _ in range(2):
        sim.step(1)
        d.step()
    got = sim.dense(L.POPS)
    sim.close()
    r = rel(got, d.f)
    print(which, "fp32 rel", r, flush=True)
    assert r < 5e-5


def _vel_rel_l2(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300)))


def test_porous32_chi16_truncated_vs_mps_oracle():
    """Truncated run (chi = 16 < full rank) on a 32^3 porous medium: FP64
    and FP32 policies against the CPU MPS oracle on the same schedule."""
    L = lib()
    case = WL.case_porous(n=5, chi=16, tol=1e-6)
    case = _case_with_flow(case)
    m = MPSLBM(case)
    sims = {p: L.Simulation(case, precision=p) for p in ("fp64", "fp32")}
    for _ in range(2):
        m.step()
        for s in sims.values():
            s.step(1)
    ref = m.dense_populations()
    out = {}
    for p, s in sims.items():
        out[p] = rel(s.dense(L.POPS), ref)
        s.close()
    print("porous32 chi16 rel vs MPS oracle", out, flush=True)
    # FP64: the rounding level of the algebra through two truncated steps
    # (3e-13 measured); FP32: storage rounding (6e-8) through some 300
    # roundings per step (2.7e-6 measured), bound about 7x that
    assert out["fp64"] < 1e-10
    assert out["fp32"] < 2e-5


def test_batched_domains_match_single_domains():
    """Three domains advanced by one handle (shared launches) give the same
    populations as three single-domain handles, and match the CPU MPS
    oracle.  (The dense oracle is not the reference here: with the paper's
    candidate, a product whose exact rank exceeds the candidate's bonds is
    not exact even at full chi, and one of these states has such products.)"""
    L = lib()
    c1 = _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13), seed=3)
    c2 = _case_with_flow(WL.case_porous(n=3, chi=64, tol=1e-13, tau=0.7), seed=5)
    c3 = _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13, tau=0.65, g=3e-6), seed=7)
    cases = [c1, c2, c3]
    b = L.BatchSimulation(cases, precision="fp64")
    assert b.domains() == 3
    singles = [L.Simulation(c, precision="fp64") for c in cases]
    refs = [MPSLBM(c) for c in cases]
    for _ in range(2):
        b.step(1)
        for s in singles:
            s.step(1)
        for m in refs:
            m.step()
    for k, c in enumerate(cases):
        got = b.dense(k)
        one = singles[k].dense()
        ref = refs[k].dense_populations()
        print(c.name, "batch vs single", rel(got, one), "vs MPS oracle", rel(got, ref), flush=True)
        assert rel(got, one) < 1e-12
        assert rel(got, ref) < 1e-10
        ob, os_ = b.observables(k), singles[k].observables()
        assert abs(ob.mass - os_.mass) <= 1e-12 * abs(os_.mass)
    for s in singles:
        s.close()
    b.close()


def test_graph_captured_step_matches_eager():
    """A captured step replayed from a HIP graph equals the eager step; each
    replay is checked, with eager work and synchronisation in between."""
    L = lib()
    case = _case_with_flow(WL.case_porous(n=4, chi=16, tol=1e-6), seed=9)
    s1, s2 = _hip_stream(), _hip_stream()
    eager = L.Simulation(case, precision="fp32", hip_stream=s1)
    graph = L.Simulation(case, precision="fp32", hip_stream=s2)
    graph.capture()  # takes one eager step
    eager.step(1)
    for k in range(4):
        eager.step(1)
        graph.step(1)
        a, b = eager.dense(), graph.dense()
        oa, ob = eager.observables(), graph.observables()
        print("replay", k, "rel", rel(b, a), flush=True)
        assert rel(b, a) < 1e-9
        assert oa.step == ob.step and oa.roundings == ob.roundings
        assert [list(r) for r in oa.bonds] == [list(r) for r in ob.bonds]
    eager.close()
    graph.close()


@pytest.mark.parametrize("which", ["porous16", "vascular16"])
def test_bf16_contraction_policy(which):
    """BF16 policy (product contractions on BF16 MFMA, FP32 elsewhere) on
    the untruncated open-face geometries: the BF16 rounding of the product
    operands (relative 2^-9) perturbs the populations at the 1e-3 level; the
    bound 1e-2 leaves room for its accumulation over two steps."""
    L = lib()
    if which == "porous16":
        case = WL.case_porous(n=4, chi=64, tol=1e-7)
    else:
        case = WL.case_vascular(n=4, chi=64, tol=1e-7)
    case = _case_with_flow(case)
    sb = L.Simulation(case, precision="bf16")
    sf = L.Simulation(case, precision="fp32")
    d = DenseLBM(case)
    for _ in range(2):
        sb.step(1)
        sf.step(1)
        d.step()
    gb, gf = sb.dense(L.POPS), sf.dense(L.POPS)
    sb.close()
    sf.close()
    print(which, "bf16 vs dense", rel(gb, d.f), "fp32 vs dense", rel(gf, d.f), flush=True)
    assert rel(gb, d.f) < 1e-2
    assert rel(gf, d.f) < 5e-5


@pytest.mark.parametrize("which", ["porous16", "vascular16"])
def test_bf16x3_contraction_policy(which):
    """BF16X3 policy (product contractions on BF16 MFMA with each FP32
    operand split into three BF16 terms): the dropped terms are of relative
    order 2^-24, so the untruncated open-face geometries stay at the FP32
    policy's bound against the dense oracle."""
    L = lib()
    if which == "porous16":
        case = WL.case_porous(n=4, chi=64, tol=1e-7)
    else:
        case = WL.case_vascular(n=4, chi=64, tol=1e-7)
    case = _case_with_flow(case)
    s3 = L.Simulation(case, precision="bf16x3")
    d = DenseLBM(case)
    for _ in range(2):
        s3.step(1)
        d.step()
    g3 = s3.dense(L.POPS)
    s3.close()
    print(which, "bf16x3 vs dense", rel(g3, d.f), flush=True)
    assert rel(g3, d.f) < 5e-5


def test_rank_predictor_randomized_truncation():
    """Rank-predicted randomized truncation (FP32 policy) on a
    tolerance-limited 32^3 flow: sketches are attempted from the second step
    on and some are accepted; every accepted truncation meets the same
    tolerance rule with its exact discarded weight, so the populations stay
    within a few tolerances of the run without the predictor."""
    L = lib()
    case = _case_with_flow(WL.case_channel(n=5, chi=64, tol=1e-5), seed=3)
    on = L.Simulation(case, precision="fp32", rank_predictor=1)
    off = L.Simulation(case, precision="fp32")
    for _ in range(3):
        on.step(1)
        off.step(1)
    a, b = on.dense(L.POPS), off.dense(L.POPS)
    o = on.observables()
    on.close()
    off.close()
    d = float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    print("attempted", o.rs_attempted, "accepted", o.rs_accepted, "rel L2 on/off", d, flush=True)
    assert o.rs_attempted > 0 and o.rs_accepted > 0
    assert d < 50 * case.tol


def test_rank_predictor_cap_bound():
    """Bonds held at chi (porous 32^3, chi 16): sketches of width 16 + 8 are
    accepted only where their discarded weight is provably within 5% of the
    optimal rank-chi truncation's, so the error against the untruncated
    dense oracle stays that of the run without the predictor."""
    L = lib()
    case = _case_with_flow(WL.case_porous(n=5, chi=16, tol=1e-6), seed=3)
    on = L.Simulation(case, precision="fp32", rank_predictor=1, rank_oversample=8)
    off = L.Simulation(case, precision="fp32")
    d = DenseLBM(case)
    for _ in range(3):
        on.step(1)
        off.step(1)
        d.step()
    a, b = on.dense(L.POPS), off.dense(L.POPS)
    o = on.observables()
    on.close()
    off.close()
    e_on = float(np.sqrt(((a - d.f) ** 2).sum() / (d.f ** 2).sum()))
    e_off = float(np.sqrt(((b - d.f) ** 2).sum() / (d.f ** 2).sum()))
    print("attempted", o.rs_attempted, "accepted", o.rs_accepted, "error vs dense: on", e_on,
          "off", e_off, flush=True)
    assert o.rs_attempted > 0
    assert e_on <= 1.5 * e_off + 1e-6


def test_porous64_full_size_step_vs_mps_oracle():
    """The benchmark configuration at its full size (64^3 porous medium,
    chi = 64, tol 1e-8, FP32 policy, the launch shapes the benchmark times),
    started from a seeded flow (|u| ~ 1e-2) so that the velocity carries
    signal: two steps against the CPU FP64 MPS oracle on the same
    schedule.  Populations, velocity (u = j / rho of the dense populations)
    and mass are compared."""
    from oracle.dense_lbm import moments
    L = lib()
    case = _case_with_flow(WL.case_porous(n=6, chi=64, tau=0.6, tol=1e-8, precision="fp32"))
    m = MPSLBM(case)
    s = L.Simulation(case)
    for _ in range(2):
        m.step()
        s.step(1)
    fr = m.dense_populations()
    fg = s.dense(L.POPS)
    s.close()
    rr, jr = moments(fr)
    rg, jg = moments(fg.astype(np.float64))
    fluid = ~np.asarray(case.solid, dtype=bool)  # velocity is defined in fluid cells
    ur, ug = jr[:, fluid] / rr[fluid], jg[:, fluid] / rg[fluid]
    du = _vel_rel_l2(ug, ur)
    df = float(np.sqrt(((fg - fr) ** 2).sum() / (fr ** 2).sum()))
    dm = abs(float(fg.sum()) - float(fr.sum())) / float(fr.sum())
    print("porous64 full size: velocity rel L2", du, "populations rel L2", df, "mass", dm,
          "|u| rms", float(np.sqrt((ur ** 2).mean())), flush=True)
    # velocity: the 1e-4 relative L2 asked of the reduced-precision step
    # against the FP64 oracle; populations and mass: FP32 storage (eps 6e-8)
    # through about 300 roundings per step, each truncating at chi, leaves
    # differences of a few 1e-6 (3e-6 and 5e-7 measured)
    assert du < 1e-4
    assert df < 1e-5
    assert dm < 1e-5


def test_predictor_network_gradient_vs_oracle():
    """Forward and backward kernels of the rank-predictor network (FP32)
    against the FP64 numpy backpropagation of the oracle on the same
    parameters and batch."""
    from oracle import mlp as M
    L = lib()
    rng = np.random.default_rng(11)
    p = np.zeros(M.NPARAM)
    off = 0
    for name, shape in M.SHAPES:
        n = int(np.prod(shape))
        p[off:off + n] = (rng.uniform(-1, 1, n) * np.sqrt(6.0 / shape[0]) if name.startswith("W")
                          else rng.uniform(-0.1, 0.1, n))
        off += n
    p = p.astype(np.float32)
    x = rng.uniform(-2, 0, (96, M.IN)).astype(np.float32)
    t = rng.normal(0, 0.5, 96).astype(np.float32)
    loss_g, grad_g = L.mps_lbm_mlp_gradient(p, x, t)
    loss_o, grad_o = M.gradient(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    rg = float(np.linalg.norm(grad_g - grad_o) / np.linalg.norm(grad_o))
    print("network loss", loss_g, loss_o, "gradient rel L2", rg, flush=True)
    assert abs(loss_g - loss_o) <= 1e-5 * max(1.0, loss_o)
    assert rg < 1e-5


def test_learned_rank_predictor_end_to_end():
    """Learned predictor on a tolerance-limited 32^3 flow: spectra recorded
    during steps train the network with the library's kernels (the loss
    falls), its ranks then size the sketches, and the state stays within a
    few tolerances of the run without the predictor; the mean rank errors of
    the network and of the previous-rank prediction are reported."""
    L = lib()
    case = _case_with_flow(WL.case_channel(n=5, chi=64, tol=1e-5), seed=3)
    on = L.Simulation(case, precision="fp32", rank_predictor=2)
    off = L.Simulation(case, precision="fp32")
    for _ in range(4):
        on.step(1)
        off.step(1)
    i0 = on.predictor_info()
    loss = on.train_predictor(150, 1e-3)
    for _ in range(2):
        on.step(1)
        off.step(1)
    i1 = on.predictor_info()
    a, b = on.dense(L.POPS), off.dense(L.POPS)
    o = on.observables()
    on.close()
    off.close()
    d = float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    print("samples", i0.samples, "loss first/last", i1.first_loss, i1.last_loss, loss,
          "predictions", i1.predictions, "mean |rank error| network", i1.mlp_abs_err,
          "previous rank", i1.prev_abs_err, "sketches", o.rs_attempted, o.rs_accepted,
          "rel L2 on/off", d, flush=True)
    assert i0.samples > 100 and i1.trained == 1
    assert i1.last_loss < 0.5 * i1.first_loss
    assert i1.predictions > 0 and o.rs_accepted > 0
    assert d < 50 * case.tol


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_split_autotuner_keeps_the_step(prec):
    """The autotuner retimes the contractions met in a step and picks their
    share counts of K (and, for the products on BF16 matrix cores, their
    tile edge); the step it then runs differs from the untuned one only by
    the summation order of the contractions whose share count changed."""
    L = lib()
    case = _case_with_flow(WL.case_porous(n=5, chi=64, tol=1e-8), seed=4)
    a = L.Simulation(case, precision=prec)
    b = L.Simulation(case, precision=prec)
    a.step(1)
    b.step(1)
    tuned = a.autotune()
    for _ in range(2):
        a.step(1)
        b.step(1)
    fa, fb = a.dense(L.POPS), b.dense(L.POPS)
    a.close()
    b.close()
    d = float(np.sqrt(((fa - fb) ** 2).sum() / (fb ** 2).sum()))
    print(prec, "classes tuned", tuned, "rel L2 tuned/untuned", d, flush=True)
    assert tuned > 0
    assert d < 1e-4


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-10), ("fp32", 5e-5)])
def test_minimum_size_4cubed(prec, bound):
    """The smallest grid (4^3, two sites per MPS: one bond, of rank at most
    8) with walls and a body force, untruncated, against the dense oracle."""
    L = lib()
    case = _case_with_flow(WL.case_channel(n=2, chi=64, tol=1e-13), seed=5)
    s = L.Simulation(case, precision=prec)
    d = DenseLBM(case)
    for _ in range(2):
        s.step(1)
        d.step()
    g = s.dense(L.POPS)
    s.close()
    print("4^3", prec, "rel vs dense", rel(g, d.f), flush=True)
    assert rel(g, d.f) < bound


def test_rest_state_rank_one_fixed_point():
    """Degenerate inputs at the benchmark's grid size: an all-fluid periodic
    64^3 box at rest (uniform density, no force, no solid cell, so the mask
    MPS is zero) held at chi = 1.  The equilibrium at rest is a fixed point
    of the step, and every MPS is rank one, so three steps must return the
    initial populations w_i with every bond at 1."""
    L = lib()
    n = 6
    N = 1 << n
    case = WL.Case(name="rest64", n=n, tau=0.8, chi=1, tol=1e-8,
                   solid=np.zeros((N, N, N), dtype=np.uint8), precision="fp32")
    s = L.Simulation(case)
    f0 = s.dense(L.POPS)
    s.step(3)
    f3 = s.dense(L.POPS)
    o = s.observables()
    s.close()
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    print("rest state: max |f3 - f0|", float(np.abs(f3 - f0).max()), "max bond", o.max_bond,
          flush=True)
    assert np.abs(np.sort(f0.reshape(19, -1).mean(axis=1)) - np.sort(w)).max() < 1e-6
    assert np.abs(f3 - f0).max() < 1e-6
    assert o.max_bond == 1


def _read_velocity_fixture(path):
    cells, u = [], []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = line.split()
        cells.append([int(t) for t in v[:3]])
        u.append([float(t) for t in v[3:]])
    return np.array(cells), np.array(u).T


def test_vascular128_full_size_velocity_vs_oracle():
    """The 128^3, chi = 128 branching-tube configuration (velocity inlet,
    pressure outlet, obstacle mask at machine precision) at full size and in
    the launch configuration the benchmark times: FP32 and BF16X3 policies,
    two steps from a seeded flow, against the CPU FP64 MPS oracle on the
    same schedule.  The oracle's velocity u = j / rho after the two steps is
    stored at 6000 seeded fluid cells (tests/golden, written by the
    committed script beside it, which calls only the oracle); the relative
    L2 difference over those cells must stay below the 1e-4 asked of the
    reduced-precision step.  Between the two steps the contraction
    autotuner runs, as in the benchmark, so that the second step uses the
    tuned split-K counts and tile edges."""
    import os
    L = lib()
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "vascular128_chi128_velocity_samples.txt")
    from oracle import mps as M
    cells, u_ref = _read_velocity_fixture(path)
    case = _case_with_flow(WL.case_vascular(n=7, chi=128, tau=0.55, tol=1e-8))
    x, y, z = cells.T
    assert not case.solid[x, y, z].any()
    mask_bond = max(M.bonds(M.from_dense(case.solid.astype(np.float64), 7, 1 << 30, 1e-12)))
    for prec in ("fp32", "bf16x3"):
        print("vascular128 chi128", prec, "two steps", flush=True)
        s = L.Simulation(case, precision=prec)
        s.step(1)
        print("vascular128", prec, "classes tuned", s.autotune(), flush=True)
        s.step(1)
        vel = s.dense(L.VEL)
        o = s.observables()
        s.close()
        du = _vel_rel_l2(vel[:, x, y, z], u_ref)
        print("vascular128", prec, "velocity rel L2 vs MPS oracle (6000 fluid cells)", du,
              "mask bond", o.mask_bond, "mask err", o.mask_trunc_err, flush=True)
        # the mask is decided in FP64 (the oracle's ranks) and stored in FP32
        assert o.mask_bond == mask_bond and o.mask_trunc_err < 1e-6
        assert du < 1e-4


def test_porous64_chi128_wide_factorisations_vs_mps_oracle():
    """64^3 porous medium at chi = 128: the sums carry bonds of 256, so the
    truncations run the factorisation paths wider than 128 columns (global
    memory Cholesky and Jacobi).  Two FP32 steps against the CPU FP64 MPS
    oracle on the same schedule."""
    from oracle.dense_lbm import moments
    L = lib()
    case = _case_with_flow(WL.case_porous(n=6, chi=128, tau=0.6, tol=1e-8, precision="fp32"))
    print("porous64 chi128 fp32: oracle two steps", flush=True)
    m = MPSLBM(case)
    for _ in range(2):
        m.step()
    fr = m.dense_populations()
    s = L.Simulation(case)
    s.step(2)
    fg = s.dense(L.POPS)
    o = s.observables()
    s.close()
    rr, jr = moments(fr)
    rg, jg = moments(fg)
    fluid = ~np.asarray(case.solid, dtype=bool)
    du = _vel_rel_l2(jg[:, fluid] / rg[fluid], jr[:, fluid] / rr[fluid])
    df = float(np.sqrt(((fg - fr) ** 2).sum() / (fr ** 2).sum()))
    print("porous64 chi128: max bond", o.max_bond, "velocity rel L2", du, "populations", df,
          flush=True)
    assert o.max_bond > 64
    assert du < 1e-4
    assert df < 1e-5


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-10), ("fp32", 5e-5)])
def test_newton_inverse_density_untruncated(prec, bound):
    """Newton-Schulz inverse density (three iterations, Appendix B) on the
    body-forced 8^3 channel, untruncated, two steps, against the CPU MPS
    oracle run in the same mode.  The reference is the MPS oracle, not the
    dense one: the Newton products act on operands of order one (rho (.) y is
    about 1), so the fitting error of the two-sweep variational product
    (about 1e-9 here) stays in the result, and only the MPS oracle runs the
    same product.  The body force makes j_eq a sum that the library rounds
    together with the first Newton sum."""
    L = lib()
    case = _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13))
    print("case", case.name, prec, "newton x3", flush=True)
    sim = L.Simulation(case, precision=prec, inv_mode=L.INV_NEWTON, inv_iters=3)
    sim.step(2)
    got = sim.dense(L.POPS)
    sim.close()
    m = MPSLBM(case, inv_mode="newton", inv_iters=3)
    m.step()
    m.step()
    r = rel(got, m.dense_populations())
    print("rel vs MPS oracle", r, flush=True)
    assert r < bound


def test_newton_inverse_density_truncated_vs_mps_oracle():
    """Newton-Schulz inverse density (two iterations) with truncation
    (chi = 8 on the body-forced 16^3 channel), FP64 and FP32 policies
    against the CPU MPS oracle on the same schedule, two steps."""
    L = lib()
    case = _case_with_flow(WL.case_channel(n=4, chi=8, tol=1e-6))
    print("case", case.name, "chi 8 newton x2", flush=True)
    m = MPSLBM(case, inv_mode="newton", inv_iters=2)
    sims = {p: L.Simulation(case, precision=p, inv_mode=L.INV_NEWTON, inv_iters=2)
            for p in ("fp64", "fp32")}
    for _ in range(2):
        m.step()
        for s in sims.values():
            s.step(1)
    ref = m.dense_populations()
    out = {}
    for p, s in sims.items():
        out[p] = rel(s.dense(L.POPS), ref)
        s.close()
    print("channel16 chi8 newton rel vs MPS oracle", out, flush=True)
    # FP64: 8.8e-13 measured.  FP32: 1.5e-4 measured: at chi 8 every
    # truncation of this flow is held at chi with closely spaced singular
    # values at the cut, where an FP32-level perturbation turns the kept
    # subspace; bound about 3x the measured value
    assert out["fp64"] < 1e-10
    assert out["fp32"] < 5e-4


def test_batched_domains_beyond_one_launch():
    """Five domains in one handle: the levels of a step then hold 90 to 245
    problems, more than one launch carries (64), so roundings, sums and
    shifts are issued in several chunks.  Each domain must still match its
    own single-domain handle and the CPU MPS oracle."""
    L = lib()
    cases = [
        _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13), seed=11),
        _case_with_flow(WL.case_porous(n=3, chi=64, tol=1e-13, tau=0.7), seed=12),
        _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13, tau=0.65, g=3e-6), seed=13),
        _case_with_flow(WL.case_porous(n=3, chi=64, tol=1e-13, tau=0.9, seed=2520), seed=14),
        _case_with_flow(WL.case_channel(n=3, chi=64, tol=1e-13, tau=0.75, g=-2e-6), seed=15),
    ]
    print("five domains", [c.name for c in cases], flush=True)
    b = L.BatchSimulation(cases, precision="fp64")
    assert b.domains() == 5
    singles = [L.Simulation(c, precision="fp64") for c in cases]
    refs = [MPSLBM(c) for c in cases]
    for _ in range(2):
        b.step(1)
        for s in singles:
            s.step(1)
        for m in refs:
            m.step()
    for k, c in enumerate(cases):
        got = b.dense(k)
        one = singles[k].dense()
        ref = refs[k].dense_populations()
        print(k, c.name, "batch vs single", rel(got, one), "vs MPS oracle", rel(got, ref), flush=True)
        assert rel(got, one) < 1e-12
        assert rel(got, ref) < 1e-10
    for s in singles:
        s.close()
    b.close()


def test_pinfin_tensor_product_mask_vs_oracle():
    """Pin array whose mask is given as a coarse layout and a unit pin
    (Appendix D): the library's chained mask has the oracle's bonds exactly
    and its entries to the storage precision, its largest bond is the larger
    of the two parts', and two truncated steps match the CPU MPS oracle on
    the same schedule.

    The FP32 policy runs at chi = 32: at chi = 16 the obstacle products of
    this state exceed the population's bond space (the candidate), and the
    fitted projection then moves with FP32 rounding to 8.6e-5 relative in
    the populations, 8.6e-4 in the velocity (measured)."""
    from oracle import mps as M
    L = lib()
    out = {}
    for p, chi in (("fp64", 16), ("fp32", 32)):
        case = _case_with_flow(WL.case_pinfin(n=5, l=3, chi=chi, tau=0.6, tol=1e-6,
                                              precision="fp64"))
        print("pinfin32 tensor mask", p, "chi", chi, flush=True)
        m = MPSLBM(case)
        if p == "fp64":
            ref_mask = M.to_dense(m.mask)
            outer, inner = case.mask_parts
            part_max = max(
                M.max_bond(M.from_dense(outer.astype(float), 3, 1 << 30, case.tol_mask)),
                M.max_bond(M.from_dense(inner.astype(float), 2, 1 << 30, case.tol_mask)))
        s = L.Simulation(case, precision=p)
        cores = s.mps(L.MPS_MASK)
        o = s.observables()
        dm = float(np.abs(M.to_dense(cores) - ref_mask).max())
        print("pinfin32", p, "mask bonds", M.bonds(cores), "vs", M.bonds(m.mask), "entry diff", dm,
              "mask err", o.mask_trunc_err, flush=True)
        bound = 1e-12 if p == "fp64" else 1e-6
        assert M.bonds(cores) == M.bonds(m.mask)
        assert o.mask_bond == part_max
        assert dm < bound and o.mask_trunc_err < bound
        # <1, m_O> from the stored mask: FP32 storage rounding (1.7e-9
        # relative measured)
        assert abs(o.n_fluid - m.n_fluid) / m.n_fluid < (1e-12 if p == "fp64" else 1e-7)
        for _ in range(2):
            m.step()
            s.step(1)
        out[p] = rel(s.dense(L.POPS), m.dense_populations())
        s.close()
    print("pinfin32 rel vs MPS oracle", out, flush=True)
    # FP64: 1.0e-12 measured; FP32 at chi 32: 7.0e-6 measured
    assert out["fp64"] < 1e-10
    assert out["fp32"] < 2e-5


def test_pinfin128_tensor_product_mask_at_full_size():
    """The 128^3 pin array (8^3 layout of 16^3 unit pins): chained mask
    bonds equal to the oracle's chain, entries to the FP64 rounding level
    against the oracle's chain, decomposition error against the composite
    at machine precision, fluid cell count exact."""
    from oracle import mps as M
    L = lib()
    case = WL.case_pinfin(n=7, l=3, chi=64, precision="fp64")
    outer, inner = case.mask_parts
    chain = M.tensor_product(M.from_dense(outer.astype(float), 3, 1 << 30, case.tol_mask),
                             M.from_dense(inner.astype(float), 4, 1 << 30, case.tol_mask))
    print("pinfin128 tensor mask init", flush=True)
    s = L.Simulation(case, precision="fp64")
    cores = s.mps(L.MPS_MASK)
    o = s.observables()
    s.close()
    dm = float(np.abs(M.to_dense(cores) - M.to_dense(chain)).max())
    print("pinfin128 mask bonds", M.bonds(cores), "entry diff", dm, "mask err",
          o.mask_trunc_err, "n_fluid", o.n_fluid, flush=True)
    assert M.bonds(cores) == M.bonds(chain)
    assert o.mask_bond == M.max_bond(chain)
    assert dm < 1e-12 and o.mask_trunc_err < 1e-12
    assert abs(o.n_fluid - float((1 - case.solid).sum())) < 1e-6


RAMP = (0.0, 1.0, 1.5, 0.0, 0.0, 0.0)        # u_0 (1 - exp(-1.5 t)), Section 4.1
PULSE = (0.1, 0.0, 0.0, 18.0, 1.5, 10.0)     # 0.1 + 18 t^1.5 exp(-10 t), Section 4.1


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-10), ("fp32", 5e-5)])
def test_profiled_inlet_untruncated_vs_dense(prec, bound):
    """Branching tube at 16^3, velocity inlet ramped as u_0 (1 - e^{-1.5 t})
    (t = 0.2 per step), untruncated, four steps against the dense oracle
    with the same profile."""
    L = lib()
    case = _case_with_flow(WL.case_vascular(n=4, chi=64, tau=0.6, u_in=0.03, tol=1e-13,
                                            precision="fp64"), seed=5)
    case.face_profile = {0: (RAMP, 0.2)}
    print("vascular16 ramped inlet", prec, flush=True)
    s = L.Simulation(case, precision=prec)
    d = DenseLBM(case)
    for _ in range(4):
        s.step(1)
        d.step()
    err = rel(s.dense(L.POPS), d.f)
    s.close()
    print("vascular16 ramped inlet", prec, "rel vs dense", err, flush=True)
    assert err < bound


def _closed_duct(n, ub, profile, dt):
    rho, u = WL.random_flow_state(n, 11, amp=0.01)
    return WL.Case(name="closed_duct", n=n, tau=0.7, chi=64, tol=1e-13,
                   axis_open=(1, 0, 0),
                   face_bc=(WL.BC_VELOCITY, WL.BC_VELOCITY, 0, 0, 0, 0),
                   face_val=((ub, 0.0, 0.0), (0.0, 0.0, 0.0)) + ((0, 0, 0),) * 4,
                   rho_init=rho, u_init=u, face_profile={0: (profile, dt)})


def test_profiled_inlet_mass_gain_and_graph_replay():
    """Closed duct (pulsed inlet on x = 0, resting velocity face on x = N-1):
    each step adds exactly N^2 rho_0 u_b phi(k dt) through the inlet (the
    identity the oracle pins), read from the library's own mass and rho_0;
    a graph-captured handle follows the profile through its replays (the
    step count lives on the device) and ends bitwise equal to the eager
    handle."""
    from oracle.inflow import inflow_scale
    L = lib()
    n, ub, dt = 4, 0.03, 0.05
    N = 1 << n
    case = _closed_duct(n, ub, PULSE, dt)
    print("closed duct pulsed inlet: eager", flush=True)
    s = L.Simulation(case, precision="fp64")
    m0 = s.observables().mass
    for k in range(5):
        s.step(1)
        o = s.observables()
        expect = N * N * o.rho0 * ub * inflow_scale(PULSE, k * dt)
        print("step", k, "mass gain", o.mass - m0, "expected", expect, flush=True)
        assert abs((o.mass - m0) - expect) < 1e-9 * abs(expect) + 1e-11
        m0 = o.mass
    eager = s.dense(L.POPS)
    s.close()
    print("closed duct pulsed inlet: graph", flush=True)
    g = L.Simulation(case, precision="fp64", hip_stream=_hip_stream())
    g.capture()            # one eager step, then the next one recorded
    for _ in range(4):
        L.load().mps_lbm_step(g.h, 1)
    got = g.dense(L.POPS)
    g.close()
    assert np.array_equal(got, eager)


def test_pressure_drop_observable_vs_oracle():
    """Delta p / p_0 over the inflow region of the 32^3 pin array (the
    region Section 4.2 uses for the pin-fin case, x < 2 N / 256 widened to
    two cells, y and z < N / 2) after three steps with the ramped inlet
    from a seeded flow, FP64 at chi 16 and FP32 at chi 32, against the
    oracle's metric on its own state; the exact fluid-cell count of the
    region.  (From rest, the paper's start, the state is symmetric across
    the pin rows and its truncations cut through degenerate singular values,
    where two FP64 implementations already keep different directions: the
    metric then differs by 1.6e-7 after three steps, measured.)"""
    from oracle.metrics import pressure_drop
    L = lib()
    lo, hi = (0, 0, 0), (2, 16, 16)
    # measured: FP64 2.0e-13, FP32 2.0e-7 against the oracle
    for p, chi, bound in (("fp64", 16, 1e-12), ("fp32", 32, 2e-6)):
        case = WL.case_pinfin(n=5, l=3, chi=chi, tau=0.6, tol=1e-6, u_in=0.03,
                              precision="fp64")
        case = _case_with_flow(case)
        case.face_profile = {0: (RAMP, 0.5)}
        print("pinfin32 pressure drop", p, "chi", chi, flush=True)
        m = MPSLBM(case)
        s = L.Simulation(case, precision=p)
        s.set_region(lo, hi, 1.0)
        for _ in range(3):
            m.step()
            s.step(1)
        o = s.observables()
        ref = m.pressure_drop(lo, hi, 1.0)
        cells = float((1 - case.solid[0:2, 0:16, 0:16]).sum())
        # the library's metric on the library's own dense density
        own = pressure_drop(s.dense(L.RHO), case.solid, lo, hi, 1.0)
        s.close()
        print("pinfin32", p, "dp/p0", o.dp_p0, "oracle", ref, "own dense", own, "cells",
              o.region_cells, "region err", o.region_trunc_err, flush=True)
        assert o.region_cells == cells
        assert o.region_trunc_err < (1e-12 if p == "fp64" else 1e-6)
        # (FP32: 3.7e-9 measured, the dense contraction runs in FP32)
        assert abs(o.dp_p0 - own) < (1e-13 if p == "fp64" else 5e-8)
        assert abs(o.dp_p0 - ref) < bound
        assert abs(ref) > 1e-6


def test_pressure_drop_observable_at_64cubed():
    """The metric's contraction at the porous 64^3 ranks (mask region of
    bond about 400 against populations of bond 64): a box in the middle of
    the medium at init, FP32, against the oracle's metric on its initial
    state."""
    L = lib()
    case = _case_with_flow(WL.case_porous(n=6, chi=64, tau=0.6, tol=1e-8, precision="fp32"),
                           amp=0.02)
    lo, hi = (20, 8, 5), (44, 50, 61)
    print("porous64 pressure drop at init", flush=True)
    m = MPSLBM(case)
    ref = m.pressure_drop(lo, hi, 1.0)
    s = L.Simulation(case)
    s.set_region(lo, hi, 1.0)
    o = s.observables()
    s.close()
    print("porous64 dp/p0", o.dp_p0, "oracle", ref, "region err", o.region_trunc_err,
          flush=True)
    # 1.7e-8 measured (FP32 storage of populations and region)
    assert abs(o.dp_p0 - ref) < 2e-7


@pytest.mark.parametrize("which", ["tgv8", "porous16"])
@pytest.mark.parametrize("prec,bound", [("fp64", 1e-10), ("fp32", 5e-5)])
def test_d3q15_untruncated_vs_dense(which, prec, bound):
    """The paper's D3Q15 velocity set (Section 4.1): the Taylor-Green vortex
    at 8^3 and the porous medium at 16^3 (pressure faces, obstacles, corner
    velocities streamed as three axis shifts), untruncated, three steps
    against the dense oracle."""
    L = lib()
    if which == "tgv8":
        case = WL.case_tgv(n=3, chi=64, re=50.0, tol=1e-14, precision="fp64")
    else:
        case = _case_with_flow(WL.case_porous(n=4, chi=64, tau=0.6, tol=1e-13,
                                              precision="fp64"), seed=5)
        case.lattice = 15
    print("d3q15", which, prec, flush=True)
    s = L.Simulation(case, precision=prec)
    d = DenseLBM(case)
    for _ in range(3):
        s.step(1)
        d.step()
    got = s.dense(L.POPS)
    o = s.observables()
    s.close()
    err = rel(got, d.f)
    print("d3q15", which, prec, "rel vs dense", err, flush=True)
    assert got.shape[0] == 15 and err < bound
    assert all(o.bonds[i][0] == 0 for i in range(15, 19))


def test_tgv32_truncated_vs_mps_oracle_and_kinetic_energy():
    """Taylor-Green vortex at 32^3 on D3Q15 (Re 800 as in Section 5.1,
    chi 16 < full rank): two truncated steps, FP64 and FP32, against the CPU
    MPS oracle; the kinetic-energy entry point against the oracle's metric
    on the library's own state and on the oracle's.  The vortex is
    symmetric, so its spectra hold equal singular values, some of them at
    the chi cut, where rounding-level differences turn the kept subspace:
    FP64 differs from the oracle by 1.4e-9 (measured), not the 1e-13 of the
    porous medium.  Under FP32 the turn is of the size of the singular
    values at the cut (2.9e-4 relative, measured), every such subspace being
    an equally valid truncation: there the test checks what is unique, the
    kinetic energy, and that the state is as close to the untruncated dense
    solution as the oracle's own truncated state is."""
    from oracle.metrics import kinetic_energy
    L = lib()
    case = WL.case_tgv(n=5, chi=16, re=800.0, tol=1e-8, precision="fp64")
    m = MPSLBM(case)
    d = DenseLBM(case)
    for _ in range(2):
        m.step()
        d.step()
    ref = m.dense_populations()
    e_ref = kinetic_energy(ref)
    l2 = lambda a, b: float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    trunc_ref = l2(ref, d.f)
    for p in ("fp64", "fp32"):
        print("tgv32 chi16", p, flush=True)
        s = L.Simulation(case, precision=p)
        s.step(2)
        f = s.dense(L.POPS)
        e = s.kinetic_energy()
        s.close()
        err = rel(f, ref)
        e_own = kinetic_energy(f)
        trunc = l2(f, d.f)
        print("tgv32", p, "rel vs MPS oracle", err, "E_kin", e, "own dense", e_own, "oracle", e_ref,
              "L2 to dense", trunc, "oracle's", trunc_ref, flush=True)
        assert abs(e - e_own) < 1e-12 * e_own
        if p == "fp64":
            assert err < 1e-8
            assert abs(e - e_ref) < 1e-10 * e_ref
        else:
            # measured: E_kin 1.1e-6 relative
            assert abs(e - e_ref) < 1e-5 * e_ref
            assert trunc < 1.5 * trunc_ref + 1e-6


def test_tgv32_kinetic_energy_decay_vs_dense():
    """The vortex's kinetic energy over 120 steps at 32^3 (D3Q15, Re 100,
    untruncated: chi at the full bond 64), FP64, every 20 steps against
    the dense oracle, and the second-order dissipation of both curves."""
    from oracle.metrics import dissipation, kinetic_energy
    L = lib()
    case = WL.case_tgv(n=5, chi=64, re=100.0, tol=1e-12, precision="fp64")
    d = DenseLBM(case)
    print("tgv32 decay: 120 steps", flush=True)
    s = L.Simulation(case, precision="fp64")
    eg, ed = [s.kinetic_energy()], [kinetic_energy(d.f)]
    for _ in range(6):
        s.step(20)
        for _ in range(20):
            d.step()
        eg.append(s.kinetic_energy())
        ed.append(kinetic_energy(d.f))
    s.close()
    eg, ed = np.array(eg), np.array(ed)
    dev = float(np.abs(eg / ed - 1).max())
    ddev = float(np.abs(dissipation(eg, 20.0) / dissipation(ed, 20.0) - 1).max())
    print("tgv32 E_kin", eg, "dense", ed, "max rel", dev, "dissipation max rel", ddev, flush=True)
    # measured: 8.2e-12 and 1.0e-10
    assert eg[-1] < 0.9 * eg[0]
    assert dev < 1e-10 and ddev < 1e-8


def test_uneven_domains_in_one_handle():
    """Domains of different sizes, bond dimensions, velocity sets and
    precisions in one handle (four groups of batched engines): after two
    steps each domain equals its own single-domain handle bitwise; a graph
    recording all groups replays bitwise like the eager handle; the FP64
    domains match the CPU MPS oracle."""
    L = lib()
    cases = [
        _case_with_flow(WL.case_porous(n=4, chi=16, tau=0.6, tol=1e-8, precision="fp64"), seed=1),
        _case_with_flow(WL.case_channel(n=5, chi=16, tau=0.7, tol=1e-8, precision="fp64"), seed=2),
        _case_with_flow(WL.case_porous(n=5, chi=8, tau=0.65, tol=1e-6, precision="fp32"), seed=3),
        _case_with_flow(WL.case_porous(n=4, chi=16, tau=0.8, tol=1e-8, precision="fp64"), seed=4),
        WL.case_tgv(n=4, chi=16, re=100.0, tol=1e-8, precision="fp32"),
    ]
    print("uneven batch of 5 (4 groups)", flush=True)
    b = L.BatchSimulation(cases)
    b.step(2)
    multi = [b.dense(d) for d in range(len(cases))]
    b.close()
    for d, c in enumerate(cases):
        s = L.Simulation(c)
        s.step(2)
        single = s.dense(L.POPS)
        s.close()
        print("domain", d, c.name, "max |multi - single|", float(np.abs(multi[d] - single).max()),
              flush=True)
        assert np.array_equal(multi[d], single)
    for d in (0, 1, 3):
        m = MPSLBM(cases[d])
        for _ in range(2):
            m.step()
        err = rel(multi[d], m.dense_populations())
        print("domain", d, "rel vs MPS oracle", err, flush=True)
        assert err < 1e-10
    print("uneven batch: graph", flush=True)
    g = L.BatchSimulation(cases, hip_stream=_hip_stream())
    e = L.BatchSimulation(cases)
    g.capture()
    e.step(1)
    for r in range(3):
        g.step(1)
        e.step(1)
        for d in range(len(cases)):
            assert np.array_equal(g.dense(d), e.dense(d)), (r, d)
    assert g.observables(2).step == 4
    g.close()
    e.close()


def test_per_domain_entry_points_of_an_uneven_handle():
    """In a handle of several groups, the per-domain calls reach the right
    domain: a velocity-face profile, a pressure region and the kinetic
    energy of domains in the second and third groups equal those of their
    single-domain handles; a constant profile (phi = 1) changes nothing."""
    L = lib()
    ramp = (0.0, 1.0, 1.5, 0.0, 0.0, 0.0)
    cases = [
        _case_with_flow(WL.case_porous(n=4, chi=16, tau=0.6, tol=1e-8, precision="fp64"), seed=1),
        _case_with_flow(WL.case_vascular(n=5, chi=16, tau=0.6, tol=1e-8, precision="fp64"), seed=2),
        _case_with_flow(WL.case_porous(n=5, chi=8, tau=0.65, tol=1e-6, precision="fp32"), seed=3),
    ]
    lo, hi = (0, 4, 4), (6, 20, 20)
    b = L.BatchSimulation(cases)
    L.mps_lbm_set_face_profile(b.h, 0, ramp, 0.3, domain=1)
    L.mps_lbm_set_region(b.h, lo, hi, 1.0, domain=2)
    b.step(3)
    got = [b.dense(d) for d in range(3)]
    e1 = L.mps_lbm_kinetic_energy(b.h, 1)
    o2 = b.observables(2)
    b.close()
    s1 = L.Simulation(cases[1])
    s1.set_face_profile(0, ramp, 0.3)
    s1.step(3)
    assert np.array_equal(got[1], s1.dense(L.POPS))
    assert e1 == s1.kinetic_energy()
    s1.close()
    s2 = L.Simulation(cases[2])
    s2.set_region(lo, hi, 1.0)
    s2.step(3)
    o = s2.observables()
    assert np.array_equal(got[2], s2.dense(L.POPS))
    assert o2.dp_p0 == o.dp_p0 and o2.region_cells == o.region_cells
    s2.close()
    # phi = 1 is the constant face, bitwise
    c = cases[1]
    a = L.Simulation(c)
    a.set_face_profile(0, (1.0, 0.0, 0.0, 0.0, 0.0, 0.0), 0.5)
    z = L.Simulation(c)
    a.step(2)
    z.step(2)
    assert np.array_equal(a.dense(L.POPS), z.dense(L.POPS))
    # clearing the profile restores the constant face from the next step on
    a.set_face_profile(0, None)
    z.step(1)
    a.step(1)
    assert np.array_equal(a.dense(L.POPS), z.dense(L.POPS))
    a.close()
    z.close()
