"""GPU multigrid solve: setup + flexible GCR to a true FP64 residual of 1e-10.

The stopping test is checked independently with the oracle's operator on the
host (paper Sec. 3: V-cycle-preconditioned flexible GCR; the bar 1e-10 is the
true residual |b - D x| / |b| in FP64).
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion, prepare_gauge, random_starts
from oracle import dwf

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec,cprec", [("f64", "f64"), ("f32", "f32"), ("f32", "f16"), ("f32", "bf16")])
def test_mg_solve_c1(cuda, prec, cprec):
    import paper_1205_2933_amd as mg
    L, Ls, mf = (4, 4, 4, 4), 8, 0.01
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    p = mg.make_mg_params((2, 2, 2, 2), 16, sweeps=1, sweep0_iters=100, sweep_iters=4, coarse_tol=0.1,
                          coarse_maxiter=200, fine_prec=prec, coarse_prec=cprec)
    print(f"setup C1 {prec}/{cprec}", flush=True)
    rep = mg.mgdwf_setup(h, p, dev(random_starts(L, Ls, 8, 21)))
    print("setup report", rep, flush=True)
    b = gaussian_fermion(L, Ls, 31)
    x = torch.zeros_like(dev(b))
    reps = mg.mgdwf_solve(h, dev(b), x, tol=1e-10, max_outer=400, restart=8)
    print("solve report", reps, flush=True)
    xs = x.cpu().numpy()
    r = b - dwf.apply_dwf(xs, U, 1.8, mf)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-10
    assert reps[0]["true_relres"] < 1e-10


def test_cgne_control(cuda):
    import paper_1205_2933_amd as mg
    L, Ls, mf = (4, 4, 4, 4), 8, 0.01
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    b = gaussian_fermion(L, Ls, 31)
    x = torch.zeros_like(dev(b))
    rep = mg.mgdwf_cgne(h, dev(b), x, tol=1e-10)
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - dwf.apply_dwf(xs, U, 1.8, mf)) / np.linalg.norm(b) < 1e-10
    # the oracle's CGNE takes the same number of iterations up to rounding (+-3%)
    from oracle import solvers
    A = dwf.DWF(U, 1.8, mf)
    _, orep = solvers.cgne(A, b, 1e-10, 5000)
    assert abs(rep["outer_iters"] - orep.iters) <= max(16, 0.03 * orep.iters)


@pytest.mark.parametrize("prec,cprec", [("f64", "f64"), ("f32", "f16")])
def test_coarse_graph_replay_is_bitwise_eager(cuda, prec, cprec):
    """The coarse solve's 8-iteration blocks and the V-cycle's launch sequences
    before and after the coarse solve, replayed as captured HIP graphs, give
    exactly the eager launches' result and operator counts: a tight coarse
    tolerance makes every V-cycle replay the block graph several times, with
    eager work and host synchronisations between the replays."""
    import paper_1205_2933_amd as mg
    L, Ls, mf = (4, 4, 4, 4), 8, 0.01
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    kw = dict(sweeps=1, sweep0_iters=100, sweep_iters=4, coarse_tol=1e-4, coarse_maxiter=200, fine_prec=prec,
              coarse_prec=cprec)
    mg.mgdwf_setup(h, mg.make_mg_params((2, 2, 2, 2), 16, coarse_graph=False, **kw), dev(random_starts(L, Ls, 8, 21)))
    b = dev(gaussian_fermion(L, Ls, 31, n=2))
    out = {}
    for graph in (False, True, True):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params((2, 2, 2, 2), 16, coarse_graph=graph, **kw))
        x = torch.zeros_like(b)
        reps = mg.mgdwf_solve(h, b, x, nrhs=2, tol=1e-10, max_outer=400, restart=8)
        # the V-cycle's three phase times are measured and fit inside the call
        for r in reps:
            assert all(t > 0.0 for t in r["phase_seconds"]), r
            assert sum(r["phase_seconds"]) < r["seconds"], r
            assert r["phase_seconds"] == reps[0]["phase_seconds"]
        out.setdefault(graph, []).append(
            (x.clone(), [(r["outer_iters"], r["fine_applies"], r["coarse_applies"]) for r in reps]))
    x0, r0 = out[False][0]
    assert r0[0][2] > 40 * r0[0][0]  # many coarse iterations per V-cycle: several graph blocks each
    for x1, r1 in out[True]:
        assert torch.equal(x0, x1)
        assert r1 == r0


def test_asymmetric_smoother_steps_with_graphs(cuda):
    """nu_pre != nu_post (paper Sec. 2 leaves nu1 and nu3 independent) with the
    V-cycle's launch sequences replayed as graphs: the solve converges and is
    bitwise the eager launches' result (regression: the two smoothers once
    shared a pointer table that had to be re-uploaded inside a capture)."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    kw = dict(sweeps=1, sweep0_iters=100, sweep_iters=4, coarse_tol=0.1, coarse_maxiter=200, nu_pre=6, nu_post=3,
              fine_prec="f32", coarse_prec="f16")
    mg.mgdwf_setup(h, mg.make_mg_params(block, 16, coarse_graph=False, **kw), dev(random_starts(L, Ls, 8, 21)))
    b = dev(gaussian_fermion(L, Ls, 31, n=2))
    out = []
    for graph in (False, True, True):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_graph=graph, **kw))
        x = torch.zeros_like(b)
        reps = mg.mgdwf_solve(h, b, x, nrhs=2, tol=1e-10, max_outer=400, restart=8)
        assert max(r["true_relres"] for r in reps) < 1e-10
        out.append((x.clone(), [(r["outer_iters"], r["fine_applies"]) for r in reps]))
    for x1, r1 in out[1:]:
        assert torch.equal(out[0][0], x1)
        assert r1 == out[0][1]


def test_fgcr_iterate_matches_oracle(cuda):
    """Six FP64 flexible-GCR steps with the two-level V-cycle, on the GPU and in
    the oracle, from the same basis and right-hand side (paper Sec. 2's
    five-step cycle, Sec. 3's outer solver): with the coarse CGNE run for a
    fixed 16 iterations on both sides (a tolerance never met) the two
    preconditioners are the same map, so the iterates agree up to rounding.
    Gram-Schmidt is classical on the GPU and modified in the oracle: equal in
    exact arithmetic."""
    import paper_1205_2933_amd as mg
    from oracle import setup as osu
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    A = dwf.DWF(U, 1.8, mf)
    V = random_starts(L, Ls, 8, 41)
    prm = osu.MGParams(block=block, nvec=16, nu_pre=4, nu_post=4, smoother="mr_normal", coarse_solver="cgne",
                       coarse_tol=1e-30, coarse_maxiter=16)
    omg = osu.MG(A, prm)
    omg.rebuild(V)
    b = gaussian_fermion(L, Ls, 31)
    from oracle import solvers
    xo, orep = solvers.gcr(A, b, 1e-30, 6, 8, M=omg.preconditioner())
    assert orep.iters == 6
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    mg.mgdwf_set_nullvecs(h, block, dev(osu.reflect_pairs(V)), 16)
    mg.mgdwf_build_coarse(h)
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, nu_pre=4, nu_post=4, coarse_tol=1e-30, coarse_maxiter=16,
                                                fine_prec="f64", coarse_prec="f64"))
    x = torch.zeros_like(dev(b))
    reps = mg.mgdwf_solve(h, dev(b), x, tol=1e-30, max_outer=6, restart=8, allow_not_converged=True)
    assert reps[0]["outer_iters"] == 6
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < 1e-9
    rg = np.linalg.norm(b - dwf.apply_dwf(xg, U, 1.8, mf)) / np.linalg.norm(b)
    assert abs(rg - orep.true_relres) < 1e-6 * orep.true_relres


@pytest.mark.parametrize("cprec", ["f16", "bf16"])
def test_persistent_coarse_solve(cuda, cprec):
    """The coarse CGNE as one persistent cooperative kernel (coarse_graph = 2)
    against the launched iterations (paper Sec. 2's coarse step): with a
    tolerance never met both run 16 iterations per V-cycle, so six FGCR steps
    agree up to the rounding of the coarse sums, which the persistent kernel
    takes in another order; it skips the launched loop's last, unused D_c^+
    apply.  With the tolerance of 0.1, tested every 8 iterations on both
    sides, it reaches 1e-10 against the oracle's D in the graph path's
    number of outer iterations (up to rounding)."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    kw = dict(sweeps=1, sweep0_iters=100, sweep_iters=4, fine_prec="f32", coarse_prec=cprec)
    mg.mgdwf_setup(h, mg.make_mg_params(block, 16, coarse_graph=False, **kw), dev(random_starts(L, Ls, 8, 21)))
    b = gaussian_fermion(L, Ls, 31, n=2)
    xs, counts = {}, {}
    for mode in (False, "persistent"):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_graph=mode, coarse_tol=1e-30,
                                                    coarse_maxiter=16, **kw))
        x = torch.zeros_like(dev(b))
        reps = mg.mgdwf_solve(h, dev(b), x, nrhs=2, tol=1e-30, max_outer=6, restart=8, allow_not_converged=True)
        xs[mode] = x
        counts[mode] = [(r["outer_iters"], r["fine_applies"], r["coarse_applies"]) for r in reps]
    print("counts", counts, flush=True)
    for (o0, f0, c0), (o1, f1, c1) in zip(counts[False], counts["persistent"]):
        assert (o0, f0) == (o1, f1) == (6, f0)
        assert c0 == 6 * 33 and c1 == 6 * 32
    rel = float(torch.linalg.norm(xs[False] - xs["persistent"]) / torch.linalg.norm(xs[False]))
    print("persistent vs launched", rel, flush=True)
    assert rel < 1e-3
    outer = {}
    for mode in (True, "persistent"):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_graph=mode, coarse_tol=0.1,
                                                    coarse_maxiter=200, **kw))
        x = torch.zeros_like(dev(b))
        reps = mg.mgdwf_solve(h, dev(b), x, nrhs=2, tol=1e-10, max_outer=400, restart=8, allow_not_converged=True)
        print("mode", mode, reps[0], flush=True)
        outer[mode] = reps[0]["outer_iters"]
        assert max(r["true_relres"] for r in reps) < 1e-10
    print("outer iterations", outer, flush=True)
    assert abs(outer[True] - outer["persistent"]) <= 8
    xh = x.cpu().numpy()
    for k in range(2):
        bk = b[k]
        r = bk - dwf.apply_dwf(xh[k], U, 1.8, mf)
        assert np.linalg.norm(r) / np.linalg.norm(bk) < 1e-10
        assert reps[k]["true_relres"] < 1e-10


# One V-cycle application M(b) against the oracle's TwoLevel (paper Sec. 2,
# the five steps), coarse CGNE fixed at 16 iterations on both sides.  FP64:
# the same map up to rounding.  FP32 fine level: unit roundoff 6e-8 through
# 2 x 4 MR steps (8 Dslash pairs with their step lengths) and the coarse
# Krylov iterations; the measured error is 8e-8, the bar 1e-5.  16-bit D_c:
# each coarse application carries the storage error of the 2^-11 (FP16) or
# 2^-8 (BF16) mantissa into the coarse correction; measured on M(b) it is
# 0.009 and 0.009 of a unit roundoff (4.5e-6 and 3.6e-5), the bar 0.1 unit
# roundoff.
VCYCLE_TOL = {("f64", "f64"): 1e-10, ("f32", "f32"): 1e-5, ("f32", "f16"): 0.1 * 2.0 ** -11,
              ("f32", "bf16"): 0.1 * 2.0 ** -8}


@pytest.mark.parametrize("prec,cprec", list(VCYCLE_TOL))
def test_vcycle_application_matches_oracle(cuda, prec, cprec):
    import paper_1205_2933_amd as mg
    from oracle import setup as osu
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    A = dwf.DWF(U, 1.8, mf)
    V = random_starts(L, Ls, 8, 41)
    prm = osu.MGParams(block=block, nvec=16, nu_pre=4, nu_post=4, smoother="mr_normal", coarse_solver="cgne",
                       coarse_tol=1e-30, coarse_maxiter=16)
    omg = osu.MG(A, prm)
    omg.rebuild(V)
    M = omg.preconditioner()
    b = gaussian_fermion(L, Ls, 31, n=2)
    want = np.stack([M(b[r]) for r in range(2)])
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    mg.mgdwf_set_nullvecs(h, block, dev(osu.reflect_pairs(V)), 16)
    mg.mgdwf_build_coarse(h)
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, nu_pre=4, nu_post=4, coarse_tol=1e-30, coarse_maxiter=16,
                                                fine_prec=prec, coarse_prec=cprec))
    z = torch.empty_like(dev(b))
    mg.mgdwf_apply_vcycle(h, dev(b), z, nrhs=2)
    got = z.cpu().numpy()
    for r in range(2):
        e = np.linalg.norm(got[r] - want[r]) / np.linalg.norm(want[r])
        print(f"V-cycle {prec}/{cprec} rhs {r}: {e:.3e}", flush=True)
        assert e < VCYCLE_TOL[(prec, cprec)]
    h.close()


def test_persistent_coarse_solve_several_sites_per_workgroup(cuda):
    """512 coarse sites (8^3x16 with 2^4 blocks) on a GPU of 256 CUs: the
    persistent coarse CGNE runs one workgroup per CU, each owning two coarse
    sites.  With the coarse CGNE fixed at 16 iterations (a tolerance never
    met) six FGCR steps agree with the launched loop's up to the rounding of
    the coarse sums (taken in another order), and the report flags no
    fallback to the launched loop."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, block = (8, 8, 8, 16), 4, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 14, ape_steps=2)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    kw = dict(sweeps=1, sweep0_iters=100, sweep_iters=4, fine_prec="f32", coarse_prec="f16")
    mg.mgdwf_setup(h, mg.make_mg_params(block, 16, coarse_graph=True, **kw), dev(random_starts(L, Ls, 8, 21)))
    b = gaussian_fermion(L, Ls, 31, n=2)
    out = {}
    for mode in (False, "persistent"):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_graph=mode, coarse_tol=1e-30,
                                                    coarse_maxiter=16, **kw))
        x = torch.zeros_like(dev(b))
        print(f"512-site solve mode={mode}", flush=True)
        reps = mg.mgdwf_solve(h, dev(b), x, nrhs=2, tol=1e-30, max_outer=6, restart=8, allow_not_converged=True)
        print("report", reps[0], flush=True)
        assert not (reps[0]["flags"] & 8)
        out[mode] = ([(r["outer_iters"], r["fine_applies"]) for r in reps], [r["coarse_applies"] for r in reps], x)
    assert out[False][0] == out["persistent"][0] == [(6, out[False][0][0][1])] * 2
    assert out[False][1] == [6 * 33] * 2 and out["persistent"][1] == [6 * 32] * 2
    rel = float(torch.linalg.norm(out[False][2] - out["persistent"][2]) / torch.linalg.norm(out[False][2]))
    print("persistent vs launched", rel, flush=True)
    assert rel < 1e-3
    h.close()


def test_persistent_barrier_timeout_is_an_error_not_a_hang(cuda):
    """A grid-barrier wait bounded at zero seconds runs out at once (the
    condition is forced from the host, every workgroup still leaves the kernel
    normally): the solve returns MGDWF_ERR_HIP with a message, and with the
    default bound restored the same handle solves again.  Where the persistent
    kernel does not apply (FP16 asked at FP64) nothing changes; where it is
    asked for an FP32 coarse store, the report's fallback bit is set."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    kw = dict(sweeps=1, sweep0_iters=100, sweep_iters=4, coarse_tol=0.1, coarse_maxiter=200, fine_prec="f32")
    mg.mgdwf_setup(h, mg.make_mg_params(block, 16, coarse_prec="f16", **kw), dev(random_starts(L, Ls, 8, 21)))
    b = dev(gaussian_fermion(L, Ls, 31))
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_graph="persistent", coarse_prec="f16", **kw))
    mg.mgdwf_set_barrier_timeout(h, 0.0)
    x = torch.zeros_like(b)
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_solve(h, b, x, tol=1e-10, max_outer=400, restart=8)
    assert e.value.status == mg.MGDWF_ERR_HIP and "barrier" in str(e.value)
    mg.mgdwf_set_barrier_timeout(h, 10.0)
    x = torch.zeros_like(b)
    reps = mg.mgdwf_solve(h, b, x, tol=1e-10, max_outer=400, restart=8)
    assert reps[0]["true_relres"] < 1e-10 and not (reps[0]["flags"] & 8)
    # an FP32 coarse store has no persistent kernel: the launched loop, flagged
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_graph="persistent", coarse_prec="f32", **kw))
    x = torch.zeros_like(b)
    reps = mg.mgdwf_solve(h, b, x, tol=1e-10, max_outer=400, restart=8)
    assert reps[0]["true_relres"] < 1e-10 and (reps[0]["flags"] & 8)
    with pytest.raises(mg.MgdwfError):
        mg.mgdwf_set_barrier_timeout(h, -1.0)
    h.close()


@pytest.mark.parametrize("prec,cprec,dirs", [("f64", "f64", 3), ("f32", "f16", 4), ("f32", "f16", 1)])
def test_smoother_with_fewer_kept_directions(cuda, prec, cprec, dirs):
    """smoother_dirs: at most `dirs` MR directions kept, added to x every `dirs`
    steps.  One V-cycle application equals the oracle's (the same tolerance as
    with all directions kept); on an adaptive setup a solve converges with
    graph replays and the handle holds less workspace than with every
    direction kept."""
    import paper_1205_2933_amd as mg
    from oracle import setup as osu
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    A = dwf.DWF(U, 1.8, mf)
    V = random_starts(L, Ls, 8, 41)
    prm = osu.MGParams(block=block, nvec=16, nu_pre=6, nu_post=5, smoother="mr_normal", coarse_solver="cgne",
                       coarse_tol=1e-30, coarse_maxiter=16)
    omg = osu.MG(A, prm)
    omg.rebuild(V)
    M = omg.preconditioner()
    b = gaussian_fermion(L, Ls, 31, n=2)
    want = np.stack([M(b[r]) for r in range(2)])
    used = {}
    for k in (0, dirs):
        h = mg.Handle(L, Ls, 1.8, mf)
        mg.mgdwf_set_gauge(h, dev(U))
        mg.mgdwf_set_nullvecs(h, block, dev(osu.reflect_pairs(V)), 16)
        mg.mgdwf_build_coarse(h)
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, nu_pre=6, nu_post=5, coarse_tol=1e-30,
                                                    coarse_maxiter=16, fine_prec=prec, coarse_prec=cprec,
                                                    smoother_dirs=k))
        z = torch.empty_like(dev(b))
        mg.mgdwf_apply_vcycle(h, dev(b), z, nrhs=2)
        got = z.cpu().numpy()
        for r in range(2):
            e = np.linalg.norm(got[r] - want[r]) / np.linalg.norm(want[r])
            print(f"V-cycle {prec}/{cprec} smoother_dirs {k} rhs {r}: {e:.3e}", flush=True)
            assert e < VCYCLE_TOL[(prec, cprec)]
        h.close()
    # a solve on an adaptive setup, with graph replays
    kw = dict(sweeps=1, sweep0_iters=100, coarse_tol=0.1, coarse_maxiter=200, nu_pre=6, nu_post=5)
    for k in (0, dirs):
        h = mg.Handle(L, Ls, 1.8, mf)
        mg.mgdwf_set_gauge(h, dev(U))
        mg.mgdwf_setup(h, mg.make_mg_params(block, 16, fine_prec="f64", coarse_prec="f64", **kw),
                       dev(random_starts(L, Ls, 8, 21)))
        mg.mgdwf_trim(h)
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, fine_prec=prec, coarse_prec=cprec, smoother_dirs=k,
                                                    **kw))
        x = torch.zeros_like(dev(b))
        reps = mg.mgdwf_solve(h, dev(b), x, nrhs=2, tol=1e-10, max_outer=400, restart=8)
        print(f"solve smoother_dirs {k}: {reps[0]['outer_iters']} outer iterations", flush=True)
        assert max(r["true_relres"] for r in reps) < 1e-10
        used[k] = mg.mgdwf_memory_bytes(h)
        h.close()
    assert used[dirs] < used[0]
