"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element,
on the same seeded inputs. The bar is relative L1 <= 1e-12; the arithmetic contract makes
the results identical bit for bit, and that is asserted as well."""
import itertools
import os

import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import assert_parity, gpu_evolve, note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu


# --------------------------------------------------------------------------- arithmetic

def test_device_division_and_sqrt_are_correctly_rounded():
    """Device '/' and sqrt equal the host's IEEE results bit for bit (random, subnormal,
    huge and near-tie inputs)."""
    torch = torch_gpu()
    import paper_1912_07645_amd.fv as fv
    note("arith")
    rng = np.random.default_rng(1)
    n = 4_000_000
    a = np.concatenate([
        rng.uniform(0, 10, n), np.exp(rng.uniform(-700, 700, n)),
        rng.uniform(0, 1, 1000) * 1e-310, np.array([1.0, 2.0, 4.0, 0.0, 1e-320, 1.7e308]),
        (1.0 + np.arange(1, 10001) * 2.0 ** -52) ** 2,
    ])
    b = np.concatenate([
        rng.uniform(0.1, 10, n), np.exp(rng.uniform(-700, 700, n)),
        rng.uniform(1, 2, 1000), np.array([3.0, 7.0, 3.0, 1.0, 3.0, 0.7]),
        1.0 + np.arange(1, 10001) * 2.0 ** -52,
    ])
    A = torch.from_numpy(a).cuda()
    Bt = torch.from_numpy(b).cuda()
    q = torch.empty_like(A)
    r = torch.empty_like(A)
    fv.fv_check_arith(A, Bt, q, r)
    qh, rh = q.cpu().numpy(), r.cpu().numpy()
    with np.errstate(over="ignore", under="ignore"):   # quotients past the range are +-inf / 0
        expect = a / b
    assert np.array_equal(qh, expect)
    assert np.array_equal(rh, np.sqrt(a))


# --------------------------------------------------------------------------- Sod (1D)

def test_sod_configuration_bitwise():
    """1D Euler Sod, N = 1024, first order, Rusanov, forward Euler, CFL 0.45, T = 0.2."""
    note("sod 1024")
    p = O.Problem(dim=1, n=(1024,), eq="euler", flux="rusanov", recon="first_order",
                  integrator="forward_euler", bc=("transmissive",))
    U0 = fi.sod_state(1024)
    R, rt, rsteps, rerr = O.evolve(p, U0, 0.2, 0.45)
    G, gt, gsteps, gerr, st = gpu_evolve(p, U0, 0.2, 0.45)
    assert st == 0 and gerr[0] == 0
    assert gsteps[0] == rsteps[0] and gt[0] == rt[0] == 0.2
    assert_parity(G, R, what="sod")


# --------------------------------------------------------------------------- all schemes

def _initial(p: O.Problem, seed):
    nz, ny, nx = p.n[2], p.n[1], p.n[0]
    if p.eq == "euler":
        return fi.random_smooth_state(seed, (nz, ny, nx), p.dim, batch=2)
    rng = np.random.default_rng(seed)
    base = fi.random_smooth_state(seed, (nz, ny, nx), p.dim, batch=2)[:, :1] - 1.0
    return np.ascontiguousarray(base * 5.0 + 0.1 * rng.standard_normal(base.shape))


SHAPES = {1: (600,), 2: (150, 20), 3: (20, 12, 9)}  # several tiles and ragged tails
COMBOS = [(d, eq, fl, rc, it) for d in (1, 2, 3)
          for eq, fl in (("euler", "rusanov"), ("euler", "hll"), ("euler", "hllc"),
                         ("burgers", "rusanov"), ("burgers", "hll"),
                         ("advection", "rusanov"), ("advection", "hll"))
          for rc in ("first_order", "muscl_minmod", "weno3")
          for it in ("forward_euler", "ssprk2", "ssprk3")]


@pytest.mark.parametrize("dim,eq,flux,recon,integ", COMBOS)
def test_every_scheme_matches_oracle(dim, eq, flux, recon, integ):
    idx = COMBOS.index((dim, eq, flux, recon, integ))
    bc = ("transmissive",) * 3 if idx % 3 == 0 else ("periodic",) * 3
    p = O.Problem(dim=dim, n=SHAPES[dim], eq=eq, flux=flux, recon=recon, integrator=integ, bc=bc,
                  vel=(0.7, -0.4, 0.3))
    U0 = _initial(p, 17 + dim)
    note("scheme", dim, eq, flux, recon, integ, bc[0])
    K = 6  # CFL steps; the oracle reports the step limit as EMAXSTEPS, fv_advance as success
    R, rt, rsteps, rerr = O.evolve(p, U0, 1e3, 0.4, max_steps=K)
    G, gt, gsteps, gerr, st = gpu_evolve(p, U0, 1e3, 0.4, max_steps=K, mode="advance")
    assert np.all(rerr == 6) and np.all(gerr == 0) and st == 0
    assert np.all(gsteps == K) and np.all(rsteps == K) and np.array_equal(gt, rt)
    assert_parity(G, R, what=f"{dim}D {eq} {flux} {recon} {integ}")


# --------------------------------------------------------------------------- Kelvin-Helmholtz

def _kh_problem(n, dim=2):
    return O.Problem(dim=dim, n=(n,) * dim, eq="euler", flux="hllc", recon="weno3",
                     integrator="ssprk3")


def test_kh_256_long_run_bitwise():
    """2D KH (WENO3 + HLLC + SSP-RK3, CFL 0.4) on 256^2 for 150 steps of a chaotic flow."""
    c, phi = fi.kh_coefficients(1912, [0])
    U0 = fi.kh2d_state(256, c, phi)
    p = _kh_problem(256)
    note("kh256 oracle")
    R, rt, rs, re = O.evolve(p, U0, 10.0, 0.4, max_steps=150)
    note("kh256 gpu")
    G, gt, gs, ge, st = gpu_evolve(p, U0, 10.0, 0.4, max_steps=150, mode="advance")
    assert rs[0] == gs[0] == 150 and ge[0] == 0
    assert gt[0] == rt[0]
    assert_parity(G, R, what="kh256")


def test_kh_1024_full_size_bitwise():
    """2D KH at the full 1024^2 size, first 3 steps, every cell compared."""
    c, phi = fi.kh_coefficients(1912, [0])
    U0 = fi.kh2d_state(1024, c, phi)
    p = _kh_problem(1024)
    note("kh1024 oracle")
    R, rt, rs, re = O.evolve(p, U0, 2.0, 0.4, max_steps=3)
    for v in range(solver_for(p).num_variants()):
        note("kh1024 gpu variant", v)
        G, gt, gs, ge, st = gpu_evolve(p, U0, 2.0, 0.4, max_steps=3, mode="advance", variant=v)
        assert gs[0] == 3 and gt[0] == rt[0]
        assert_parity(G, R, what=f"kh1024 variant {v}")


def test_kh3d_small_bitwise():
    cx, px, cz, pz = fi.kh3d_coefficients(1914, [0])
    U0 = fi.kh3d_state(40, cx, px, cz, pz)
    p = _kh_problem(40, dim=3)
    note("kh3d 40 oracle")
    R, rt, rs, re = O.evolve(p, U0, 10.0, 0.4, max_steps=12)
    for v in range(solver_for(p).num_variants()):
        note("kh3d 40 gpu variant", v)
        G, gt, gs, ge, st = gpu_evolve(p, U0, 10.0, 0.4, max_steps=12, mode="advance", variant=v)
        assert gs[0] == 12 and gt[0] == rt[0]
        assert_parity(G, R, what=f"kh3d variant {v}")


def test_2d_hot_variants_ragged_transmissive_batched():
    """2D WENO3 + HLLC on a ragged 70 x 83 grid with transmissive boundaries, a batch of four
    samples: every tile variant (16 x 15 and 32 x 15 tiles, each LDS plan; the last tile row and
    column end inside the grid) equals the oracle bit for bit."""
    p = O.Problem(dim=2, n=(70, 83), eq="euler", flux="hllc", recon="weno3",
                  integrator="ssprk3", bc=("transmissive",) * 3)
    U0 = np.concatenate([_initial(p, 41 + b) for b in range(2)])
    note("2d ragged oracle")
    R, rt, rs, re = O.evolve(p, U0, 1e3, 0.4, max_steps=5)
    for v in range(solver_for(p).num_variants()):
        note("2d ragged gpu variant", v)
        G, gt, gs, ge, st = gpu_evolve(p, U0, 1e3, 0.4, max_steps=5, mode="advance", variant=v)
        assert np.all(gs == 5) and np.array_equal(gt, rt)
        assert_parity(G, R, what=f"2d ragged variant {v}")


def test_3d_hot_variants_ragged_transmissive_batched():
    """3D WENO3 + HLLC on a ragged 37 x 19 x 45 grid with transmissive boundaries, a batch of
    six samples: every tile variant (cube tiles and z-marching column blocks, whose x, y
    and z extents all end inside a tile here) equals the oracle bit for bit."""
    p = O.Problem(dim=3, n=(37, 19, 45), eq="euler", flux="hllc", recon="weno3",
                  integrator="ssprk3", bc=("transmissive",) * 3)
    U0 = np.concatenate([_initial(p, 31 + b) for b in range(3)])
    note("3d ragged oracle")
    R, rt, rs, re = O.evolve(p, U0, 1e3, 0.4, max_steps=5)
    for v in range(solver_for(p).num_variants()):
        note("3d ragged gpu variant", v)
        G, gt, gs, ge, st = gpu_evolve(p, U0, 1e3, 0.4, max_steps=5, mode="advance", variant=v)
        assert np.all(gs == 5) and np.array_equal(gt, rt)
        assert_parity(G, R, what=f"3d ragged variant {v}")


# --------------------------------------------------------------------------- batching

def test_batched_equals_per_sample_and_oracle():
    """A batch of KH samples (per-sample dt) equals per-sample launches bit for bit."""
    B, n = 6, 64
    c, phi = fi.kh_coefficients(1912, np.arange(B))
    U0 = fi.kh2d_state(n, c, phi)
    p = _kh_problem(n)
    note("batch gpu")
    G, gt, gs, ge, st = gpu_evolve(p, U0, 0.15, 0.4)
    assert st == 0
    note("batch oracle")
    R, rt, rs, re = O.evolve(p, U0, 0.15, 0.4)
    assert np.array_equal(gs, rs)
    assert_parity(G, R, what="batch vs oracle")
    s = solver_for(p)
    for b in (0, 3, 5):
        note("batch single", b)
        Gb, *_ = gpu_evolve(p, U0[b:b + 1], 0.15, 0.4, solver=s)
        assert np.array_equal(Gb[0], G[b])


def test_run_to_run_graph_and_chunk_invariance():
    c, phi = fi.kh_coefficients(1912, [1])
    U0 = fi.kh2d_state(96, c, phi)
    p = _kh_problem(96)
    note("repeat a")
    A, *_ = gpu_evolve(p, U0, 0.1, 0.4)
    note("repeat b")
    Bv, *_ = gpu_evolve(p, U0, 0.1, 0.4)
    assert np.array_equal(A, Bv)
    old = {k: os.environ.get(k) for k in ("FV_NO_GRAPH", "FV_CHUNK")}
    try:
        os.environ["FV_NO_GRAPH"] = "1"
        note("eager")
        E, *_ = gpu_evolve(p, U0, 0.1, 0.4)
        os.environ.pop("FV_NO_GRAPH")
        os.environ["FV_CHUNK"] = "3"
        note("chunk 3")
        Cc, *_ = gpu_evolve(p, U0, 0.1, 0.4)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    assert np.array_equal(A, E) and np.array_equal(A, Cc)


def test_kernel_timing_counts_and_leaves_results_unchanged():
    """fv_profile_enable: the timed (eagerly enqueued) run gives the same state bit for bit,
    and the counters report the stage launches, three per enqueued SSP-RK3 step."""
    from paper_1912_07645_amd import fv
    torch = torch_gpu()
    c, phi = fi.kh_coefficients(1912, [2])
    U0 = fi.kh2d_state(64, c, phi)
    p = _kh_problem(64)
    note("profile reference")
    A, at, ak, *_ = gpu_evolve(p, U0, 0.05, 0.4)
    s = solver_for(p)
    fv.fv_profile_enable(s.handle, True)
    note("profile timed")
    T, tt, tk, *_ = gpu_evolve(p, U0, 0.05, 0.4, solver=s)
    ms, launches = fv.fv_profile_read(s.handle)
    fv.fv_profile_enable(s.handle, False)
    assert np.array_equal(A, T) and np.array_equal(at, tt) and np.array_equal(ak, tk)
    # steps are enqueued in chunks of 16, so up to 15 launches per stage past the last step
    # (which return at once) are counted too
    k = int(tk[0])
    assert launches % 3 == 0 and 3 * k <= launches < 3 * (k + 16) and ms > 0.0
    assert fv.fv_profile_read(s.handle) == (0.0, 0)


# --------------------------------------------------------------------------- failures

def test_failure_codes_match_oracle():
    torch = torch_gpu()
    p = O.Problem(dim=1, n=(300,), eq="euler", flux="hll", recon="muscl_minmod",
                  integrator="ssprk2", bc=("transmissive",))
    U0 = np.concatenate([fi.sod_state(300)] * 3)
    U0[1, 0, 0, 0, 7] = -1.0           # sample 1 starts non-physical
    note("fail codes")
    R, rt, rs, re = O.evolve(p, U0, 0.1, 0.45, max_steps=40)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 0.1, 0.45, max_steps=40)
    assert list(re) == list(ge) and re[1] == 5 and re[0] == 6
    assert np.array_equal(gs, rs)
    assert_parity(G, R, what="fail codes")
    s = solver_for(p)
    U = torch.from_numpy(U0[[0]].copy()).cuda()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = s.evolve_fixed_dt(U, 1.0, 3, cfl_bound=0.5, err=err)
    assert st == 7 and int(err[0]) == 7


def test_fixed_dt_matches_oracle():
    torch = torch_gpu()
    c, phi = fi.kh_coefficients(1915, np.arange(3))
    U0 = fi.kh2d_state(64, c, phi)
    p = O.Problem(dim=2, n=(64, 64), eq="euler", flux="rusanov", recon="muscl_minmod",
                  integrator="ssprk3")
    M, bad = O.max_speed(p, U0[0])
    dt = 0.4 / M
    note("fixed dt")
    R, re = O.evolve_fixed_dt(p, U0, dt, 25, 0.6)
    s = solver_for(p)
    U = torch.from_numpy(U0).cuda()
    err = torch.zeros(3, dtype=torch.int32, device="cuda")
    st = s.evolve_fixed_dt(U, dt, 25, 0.6, err)
    assert st == 0 and np.all(re == 0)
    assert_parity(U.cpu().numpy(), R, what="fixed dt")


# --------------------------------------------------------------------------- statistics

def test_statistics_match_oracle():
    torch = torch_gpu()
    from paper_1912_07645_amd import Stats
    B, n, H = 70, 48, 12
    c, phi = fi.kh_coefficients(1912, np.arange(B))
    U0 = fi.kh2d_state(n, c, phi)
    p = _kh_problem(n)
    note("stats evolve")
    G, *_ = gpu_evolve(p, U0, 0.05, 0.4)
    s = solver_for(p)
    st = Stats(s, max_h=H)
    Ug = torch.from_numpy(G).cuda()
    st.accumulate(Ug[:50])
    st.accumulate(Ug[50:])
    out = st.read()
    ref = O.Stats(p, max_h=H)
    ref.accumulate(G[:50])
    ref.accumulate(G[50:])
    assert out["count"] == ref.n == B
    assert_parity(out["mean"].cpu().numpy(), ref.mean, what="mean")
    assert_parity(out["var"].cpu().numpy(), ref.variance(), what="var")
    assert_parity(out["s2_mean"].cpu().numpy(), ref.s2(), bitwise=False, what="S2 mean")
    assert_parity(out["s2_var"].cpu().numpy(), ref.s2_variance(), tol=1e-10, bitwise=False,
                  what="S2 var")


@pytest.mark.parametrize("dim,n,eq,H,B", [
    (1, (37,), "advection", 20, 9),       # one line; segments end inside it; lags past n/2
    (2, (29, 19), "euler", 18, 70),       # ragged along x and y, lags up to n_y - 1, two chunks
    (3, (12, 10, 9), "euler", 8, 5),      # all three axes
    (2, (16, 24), "burgers", 15, 3),      # whole segments, a scalar field
    # lags above 64: the general kernel, reading the quantities the Welford pass writes
    (2, (130, 70), "euler", 69, 6),
    (1, (150,), "burgers", 100, 3),
])
def test_structure_functions_match_oracle(dim, n, eq, H, B):
    """Mean and variance of the quantities, and S_q(h) for h = 1..H with its moments over
    samples, against the oracle, on grids whose lines end inside a segment, lags up to n - 1
    on the shortest axis, every dimension; lags up to 64 run on the staged kernels (which form
    the quantities from the state), longer ones on the general kernel."""
    torch = torch_gpu()
    from paper_1912_07645_amd import Stats
    p = O.Problem(dim=dim, n=n, eq=eq, flux="rusanov", recon="first_order",
                  integrator="forward_euler", vel=(0.7, -0.4, 0.3))
    U0 = np.concatenate([_initial(p, 50 + b) for b in range((B + 1) // 2)])[:B]
    note("structure functions", dim, n, eq, H, B)
    st = Stats(solver_for(p), max_h=H)
    st.accumulate(torch.from_numpy(np.ascontiguousarray(U0)).cuda())
    out = st.read()
    ref = O.Stats(p, max_h=H)
    ref.accumulate(U0)
    assert out["count"] == ref.n == B
    assert_parity(out["mean"].cpu().numpy(), ref.mean, what="mean")
    if B > 1:
        assert_parity(out["var"].cpu().numpy(), ref.variance(), what="var")
    assert_parity(out["s2_mean"].cpu().numpy(), ref.s2(), bitwise=False, what="S2 mean")
    if B > 1:
        assert_parity(out["s2_var"].cpu().numpy(), ref.s2_variance(), tol=1e-10, bitwise=False,
                      what="S2 var")


def test_kh3d_full_size_sampled_cells():
    """3D KH at the full 512^3 size (one GPU's periodic subdomain, 5.4 GB per state): one
    full SSP-RK3 step on the GPU; sampled cells are recomputed by the oracle one by one from
    their 13^3 neighbourhood (after three stages a cell depends on cells within 6 of it)."""
    torch = torch_gpu()
    n = 512
    cx, px, cz, pz = fi.kh3d_coefficients(1914, [0])
    note("kh3d 512 build input")
    U0 = fi.kh3d_state(n, cx, px, cz, pz)
    p = _kh_problem(n, dim=3)
    M, bad = O.max_speed(p, U0[0])
    assert not bad
    dt = 0.4 / M
    rng = np.random.default_rng(3)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, n // 4, 7), (3, 255, 500),
           (15, 14, 31), (16, 15, 32), (31, 6, 63), (32, 7, 64)]   # tile and segment edges
    pts += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(20)]
    r = 6
    h = 2 * r + 1
    pb = O.Problem(dim=3, n=(h, h, h), eq="euler", flux="hllc", recon="weno3",
                   integrator="ssprk3", hi=(h / n, h / n, h / n))
    refs = {}
    for (i, j, kz) in pts:
        idx = [(np.arange(c - r, c + r + 1) % n) for c in (kz, j, i)]
        block = U0[0][:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]
        refs[(i, j, kz)] = O.step(pb, block, dt)[:, r, r, r]
    s = solver_for(p)
    for v in range(s.num_variants()):
        s.set_variant(v)
        U = torch.from_numpy(U0).to("cuda")
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        k = torch.zeros(1, dtype=torch.int64, device="cuda")
        note("kh3d 512 gpu step, variant", v)
        st = s.advance(U, t, 10.0, 0.4, 1, k)
        assert st == 0 and int(k[0]) == 1 and float(t[0]) == dt
        got = {q: U[0, :, q[2], q[1], q[0]].cpu().numpy() for q in pts}
        del U
        torch.cuda.empty_cache()
        for q in pts:
            assert np.array_equal(got[q], refs[q]), (v, q, got[q], refs[q])


def test_tuner_choice_keeps_parity():
    c, phi = fi.kh_coefficients(1912, [2])
    U0 = fi.kh2d_state(128, c, phi)
    p = _kh_problem(128)
    torch = torch_gpu()
    s = solver_for(p)
    Ut = torch.from_numpy(U0).cuda()
    note("tune")
    v = s.tune(Ut, reps=1)
    assert 0 <= v < s.num_variants()
    assert np.array_equal(Ut.cpu().numpy(), U0)   # the tuner leaves the state alone
    R, rt, rs, re = O.evolve(p, U0, 10.0, 0.4, max_steps=20)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 10.0, 0.4, max_steps=20, mode="advance", solver=s)
    assert_parity(G, R, what="tuned")


# --------------------------------------------------------------------------- multilevel MC

def _mlmc_oracle(ns, Ms, groups, t_end, cfl, scheme):
    """The oracle's multilevel run: every group evolved, level statistics, combination."""
    probs = [O.Problem(dim=2, n=(n, n), eq="euler", **scheme) for n in ns]
    outs = [O.evolve(p, U, t_end, cfl) for p, U in zip(probs, groups)]
    states = [o[0] for o in outs]
    levels = []
    for l, p in enumerate(probs):
        if l == 0:
            lv = O.LevelStats(p)
            lv.accumulate(states[0][:Ms[0]])
        else:
            lv = O.LevelStats(p, probs[l - 1])
            lv.accumulate(states[l][:Ms[l]], states[l - 1][Ms[l - 1]:Ms[l - 1] + Ms[l]])
        levels.append(lv)
    return states, [o[2] for o in outs], levels, O.mlmc_combine(levels)


MLMC_SCHEME = dict(flux="hll", recon="muscl_minmod", integrator="ssprk2")


def test_mlmc_pipeline_matches_oracle():
    torch = torch_gpu()
    from paper_1912_07645_amd.mlmc import MultilevelRun
    ns, Ms, T = (16, 32, 64), (24, 8, 4), 0.1
    groups = fi.mlmc_inputs(ns, Ms, seed=1913)
    note("mlmc oracle")
    R, rsteps, rlevels, rest = _mlmc_oracle(ns, Ms, groups, T, 0.4, MLMC_SCHEME)
    run = MultilevelRun(ns, Ms, dim=2, eq="euler", **MLMC_SCHEME)
    for v in range(run.solvers[0].num_variants()):
        note("mlmc gpu, variant", v)
        for s in run.solvers:
            s.set_variant(v)
        G = [torch.from_numpy(g).cuda() for g in groups]
        st, ts, errs = run.evolve(G, T, 0.4)
        assert st == 0
        est, levels = run.statistics(G)
        for l in range(3):
            assert_parity(G[l].cpu().numpy(), R[l], what=f"mlmc group {l}, variant {v}")
            out = levels[l].read()
            assert out["count"] == Ms[l]
            assert_parity(out["mean"].cpu().numpy(), rlevels[l].mean, what=f"level {l} mean")
            assert_parity(out["var"].cpu().numpy(), rlevels[l].variance(), what=f"level {l} var")
        assert_parity(est.cpu().numpy(), rest, what="mlmc estimate")
    G = [torch.from_numpy(g).cuda() for g in groups]
    v = run.tune(G, 0.4, steps=2, reps=1)
    assert 0 <= v < run.solvers[0].num_variants()
    assert all(s.tile()[1] == v for s in run.solvers)
    for l in range(3):   # tuning works on copies
        assert np.array_equal(G[l].cpu().numpy(), groups[l])


def test_multi_group_launch_equals_separate_launches():
    torch = torch_gpu()
    from paper_1912_07645_amd.mlmc import MultilevelRun
    ns, Ms, T = (16, 32, 64), (6, 3, 2), 0.05
    groups = fi.mlmc_inputs(ns, Ms, seed=7)
    run = MultilevelRun(ns, Ms, dim=2, eq="euler", **MLMC_SCHEME)
    G = [torch.from_numpy(g).cuda() for g in groups]
    note("multi group")
    run.evolve(G, T, 0.4)
    for l, n in enumerate(ns):
        p = O.Problem(dim=2, n=(n, n), eq="euler", **MLMC_SCHEME)
        note("single group", l)
        S, *_ = gpu_evolve(p, groups[l], T, 0.4)
        assert np.array_equal(S, G[l].cpu().numpy())


def test_mlmc_full_configuration_sampled():
    """The full mixed batch: 64^2/128^2/256^2/512^2 with 4096/1024/256/64 samples, MUSCL-minmod
    + HLL + SSP-RK2, CFL 0.4, T = 1. Samples of the two coarsest grids are checked against the
    oracle; every sample reaches T with positive density and conserved mass."""
    torch = torch_gpu()
    from paper_1912_07645_amd.mlmc import MultilevelRun
    ns, Ms, T = (64, 128, 256, 512), (4096, 1024, 256, 64), 1.0
    note("mlmc full build inputs")
    groups = fi.mlmc_inputs(ns, Ms, seed=1913)
    run = MultilevelRun(ns, Ms, dim=2, eq="euler", **MLMC_SCHEME)
    G = [torch.from_numpy(g).cuda() for g in groups]
    mass0 = [g[:, 0].sum(axis=(1, 2, 3)) for g in groups]
    note("mlmc full tune")
    run.tune(G, 0.4)   # the variant the benchmark runs
    note("mlmc full gpu, variant", run.solvers[0].tile()[1])
    st, ts, errs = run.evolve(G, T, 0.4)
    assert st == 0 and all(bool((t == T).all()) for t in ts)
    est, levels = run.statistics(G)
    assert torch.isfinite(est).all()
    for l in range(4):
        Gl = G[l].cpu().numpy()
        assert Gl[:, 0].min() > 0
        assert np.allclose(Gl[:, 0].sum(axis=(1, 2, 3)), mass0[l], rtol=1e-12)
    for l, idx in ((0, [0, 4095, 4096 + 1023]), (1, [0])):
        p = O.Problem(dim=2, n=(ns[l], ns[l]), eq="euler", **MLMC_SCHEME)
        note("mlmc full oracle", l, idx)
        R, *_ = O.evolve(p, groups[l][idx], T, 0.4)
        assert_parity(G[l][idx].cpu().numpy(), R, what=f"mlmc full group {l}")
