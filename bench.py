"""Benchmark: seconds per right-hand side to |b - D x| / |b| < 1e-10 (FP64 true
residual) for the domain-wall operator on a 16^3 x 32 x Ls=16 lattice at
m_f = 0.001, with the two-level adaptive multigrid of the library.

One step = one mixed-precision multi-RHS solve of the 12 spin-colour point
sources (FP32 fine level and coarse level inside the V-cycle, FP64 flexible
GCR refinement).  The FP64 plain-MG time per RHS, the Dslash bandwidth and the
setup time are measured in the same run.  Inputs are synthetic and seeded:
SU(3) links U = exp(i 0.3 H) smoothed by two APE-style steps (seed 12),
near-null starts seed 21.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

L = (16, 16, 16, 32)
L_MAIN = L
LS = 16
M5 = 1.8
MF = 0.001
BLOCK = (4, 4, 4, 4)
NVEC = 24
HBM_PEAK_GBS = 8000.0


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "dslash_f32_16c32x16_nrhs12_counters.md")
DSLASH_SRC = os.path.join(ROOT, "paper_1205_2933_amd", "csrc", "dslash.hip")


def counted_traffic(tiling_id):
    """HBM bytes per launch of the FP32 Dslash at 12 RHS, from the committed
    FETCH_SIZE / WRITE_SIZE counter summary -- or None when the kernel source
    has changed since the counters were taken, or when the autotuner picked
    another tiling than the one the counters were taken on."""
    import hashlib
    try:
        fields = dict(line.split(":", 1) for line in open(COUNTER_SUMMARY) if line.startswith("- ") and ":" in line)
        fields = {k[2:].strip(): v.strip().strip("`") for k, v in fields.items()}
        src = hashlib.sha256(open(DSLASH_SRC, "rb").read()).hexdigest()
        if fields.get("dslash.hip sha256") != src or int(fields.get("tiling id", -1)) != tiling_id:
            return None
        return float(fields["traffic bytes per launch"])
    except (OSError, KeyError, ValueError):
        return None


def dslash_kernel_name(flags):
    """The FP32 Dslash kernel a tiling's MGDWF_TILE_* flags select."""
    if flags & 64:
        return "k_dslash_tx" + (" (LDS exchange, links copied to LDS a slice ahead)" if flags & 256 else
                                " (LDS exchange)")
    if flags & 32:
        return "k_dslash_ws (wavefront per site pair)"
    if flags & 16:
        return "k_dslash_tw (t-march, pipelined)"
    return "k_dslash_tq (t-march)" if not flags & 1 else "k_dslash_tp (t-march, reloads)"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def mem(tag):
    """Device memory in use (driver view) and held by torch's allocator."""
    import torch
    free, total = torch.cuda.mem_get_info()
    log(f"[mem {tag}] used {(total - free) / 2**30:.1f} GiB of {total / 2**30:.1f}, "
        f"torch reserved {torch.cuda.memory_reserved() / 2**30:.1f} GiB")


SWEEP0_CHECK = 25  # sweep 0 keeps each vector's best iterate, checked every 25 CG iterations


def mg_params(mg, fine, coarse, coarse_graph=True):
    return mg.make_mg_params(BLOCK, NVEC, sweeps=1, sweep0_iters=400, sweep_iters=4, nu_pre=12, nu_post=12,
                             coarse_tol=0.1, coarse_maxiter=400, fine_prec=fine, coarse_prec=coarse,
                             coarse_graph=coarse_graph, sweep0_check=SWEEP0_CHECK)


def cpu_baseline(counts, x_mixed, b_mixed):
    """Oracle (numpy FP64) per-operation times on this host, combined with the GPU
    run's per-RHS operation counts into seconds per RHS solve (extrapolated).
    The oracle's Dslash is timed on the first mixed-precision solution of the
    timed step, which also gives the oracle's own |b - D x| / |b| of that GPU
    solution at the production shape."""
    import numpy as np

    from inputs import gaussian_fermion, random_starts
    from oracle import coarse as oc
    from oracle import dwf
    from oracle import transfer as ot

    cpu0, wall0 = time.process_time(), time.perf_counter()
    U = prepare_main_gauge()
    t = time.perf_counter()
    Dx = dwf.apply_dwf(x_mixed, U, M5, MF)
    t_dslash = time.perf_counter() - t
    oracle_relres = float(np.linalg.norm(b_mixed - Dx) / np.linalg.norm(b_mixed))
    del Dx
    # R and P are block local: time them on one eighth of the lattice (16^3 x 4) and scale by 8
    Ls_ = (16, 16, 16, 4)
    V = random_starts(Ls_, LS, NVEC, 21)
    x = gaussian_fermion(Ls_, LS, 2)
    Vh = V  # R and P cost the same on any basis of this shape
    t = time.perf_counter()
    c = ot.restrict(x, Vh, BLOCK)
    t_r = (time.perf_counter() - t) * 8
    t = time.perf_counter()
    ot.prolong(c, Vh, BLOCK)
    t_p = (time.perf_counter() - t) * 8
    del V, x, Vh
    Lc = tuple(L[m] // BLOCK[m] for m in range(4))
    rng = np.random.default_rng(3)
    Dc = rng.standard_normal(Lc[::-1] + (9, 2 * NVEC, 2 * NVEC)) + 0j
    cv = rng.standard_normal(Lc[::-1] + (2, NVEC)) + 0j
    t = time.perf_counter()
    oc.apply_coarse(cv, Dc)
    t_c = time.perf_counter() - t
    per_rhs = (counts["fine"] * t_dslash + counts["vcycles"] * (t_r + t_p) + counts["coarse"] * t_c)
    # threads actually used: process CPU time over wall time of the sample
    cores = max(1, round((time.process_time() - cpu0) / (time.perf_counter() - wall0)))
    return {
        "value": per_rhs, "unit": "s per RHS to 1e-10 (extrapolated)", "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle Dslash at full size ({t_dslash:.2f} s), R/P on a 16^3x4x16 slab x8 ({t_r:.2f}/{t_p:.2f} s), "
                   f"coarse apply ({t_c:.3f} s), times the GPU per-RHS counts: {counts['fine']} D applications, "
                   f"{counts['vcycles']} V-cycles, {counts['coarse']} coarse applications"),
        "oracle_check": {"true_relres_of_gpu_solution": oracle_relres,
                         "note": "|b - D x| / |b| of the first mixed-precision solution of the timed step, "
                                 "D applied by the oracle (FP64, numpy) on the host"},
    }


def prepare_main_gauge():
    from inputs import prepare_gauge
    return prepare_gauge(L, 0.3, 12, ape_steps=2)


def ragged_leg(mg, h_main, B_main, log):
    """48 solves over three lattices of uneven size in one mgdwf_solve_batch
    call: 8^4 x 8 with 20 RHS (12 point sources + 8 Gaussian), 12^3 x 24 x 12
    with 16 (12 + 4), and the main 16^3 x 32 x 16 lattice with its 12 point
    sources; mixed precision, tol 1e-10."""
    import numpy as np
    import torch

    from inputs import gaussian_fermion, point_sources, prepare_gauge, random_starts

    hs, bs = [], []
    # Ls = 12 needs a longer sweep 0: after 400 CG iterations the outer solve
    # stagnates near 5e-4, after 1000 the 16-RHS solve still misses 1e-10 in 400
    # outer iterations, after 2000 it converges in 56
    for L, Ls, seed, sweep0, ng in [((8, 8, 8, 8), 8, 14, 400, 8), ((12, 12, 12, 24), 12, 15, 2000, 4)]:
        U = prepare_gauge(L, 0.3, seed, ape_steps=2)
        h = mg.Handle(L, Ls, M5, MF, stream=torch.cuda.Stream())
        mg.mgdwf_set_gauge(h, torch.from_numpy(U).cuda())
        p_setup = mg_params(mg, "f64", "f64")
        p_setup.sweep0_iters = sweep0
        mg.mgdwf_setup(h, p_setup, torch.from_numpy(random_starts(L, Ls, NVEC // 2, 21)).cuda())
        mg.mgdwf_tune(h, nrhs=12 + ng, iters=5)
        mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "f16"))
        b = np.concatenate([point_sources(L, Ls), gaussian_fermion(L, Ls, 33, n=ng)])
        hs.append(h)
        bs.append(torch.from_numpy(b).cuda())
        mem(f"ragged, lattice {L} ready")
    # the main lattice takes its 12 point sources: its 12-RHS workspaces are
    # already allocated (16 RHS on it next to the others would need ~220 GiB)
    mg.mgdwf_set_mg_params(h_main, mg_params(mg, "f32", "f16"))  # the FP64 comparison left FP64 in place
    hs.append(h_main)
    bs.append(B_main)
    xs = [torch.zeros_like(b) for b in bs]
    nrhs = [20, 16, 12]
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    mem("ragged, before the batch")
    log("handle bytes " + ", ".join(f"{mg.mgdwf_memory_bytes(h) / 2**30:.1f} GiB" for h in hs))
    t = time.perf_counter()
    reps = mg.mgdwf_solve_batch(hs, bs, xs, nrhs, tol=1e-10, max_outer=400, restart=8, allow_not_converged=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    lat = np.array([r["seconds"] for rs in reps for r in rs])
    res = [max(r["true_relres"] for r in rs) for rs in reps]
    mem("ragged, after the batch")
    log("handle bytes " + ", ".join(f"{mg.mgdwf_memory_bytes(h) / 2**30:.1f} GiB" for h in hs))
    for h in hs[:2]:
        h.close()
    del xs, bs
    mg.mgdwf_trim(h_main)
    torch.cuda.empty_cache()
    out = {"solves": int(sum(nrhs)), "wall_s": wall, "solves_per_s": sum(nrhs) / wall,
           "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
           "outer_iters": [max(r["outer_iters"] for r in rs) for rs in reps], "max_true_relres": res,
           "lattices": ["8^4x8 (20 RHS)", "12^3x24x12 (16 RHS, sweep 0 of 2000 iterations)", "16^3x32x16 (12 RHS)"]}
    log(f"ragged batch {out}")
    assert max(res) < 1e-10, res
    return out


SQ_NVEC, SQ_SWEEP0, SQ_NU, SQ_CTOL = 24, 200, 5, 0.3


def sq_params(mg, fine, coarse):
    """The squared-operator multigrid (the paper's own): 24 adaptive vectors
    (48 coarse dof per site), 5 + 5 MR steps on D^+D, coarse CG to 0.3."""
    return mg.make_mg_params(BLOCK, SQ_NVEC, sweeps=1, sweep0_iters=SQ_SWEEP0, nu_pre=SQ_NU, nu_post=SQ_NU,
                             coarse_tol=SQ_CTOL, coarse_maxiter=400, fine_prec=fine, coarse_prec=coarse, squared=True)


def squared_leg(mg, U_dev, B_main, log):
    """The multigrid on the squared operator D^+D that the paper ran: A_c =
    P^+ D^+D P (33-point), MR smoothing on D^+D, CG on A_c, preconditioning the
    same FP64-refined flexible GCR on D x = b.  Setup from random starts, then
    one warm-up and one timed 12-RHS mixed-precision step (FP32 fine and
    coarse level), and one FP64 single-RHS solve."""
    import torch

    from inputs import random_starts

    h = mg.Handle(L_MAIN, LS, M5, MF)
    mg.mgdwf_set_gauge(h, U_dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    srep = mg.mgdwf_setup(h, sq_params(mg, "f64", "f64"), torch.from_numpy(random_starts(L_MAIN, LS, SQ_NVEC, 21)).cuda())
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    mg.mgdwf_set_mg_params(h, sq_params(mg, "f32", "f32"))
    X = torch.zeros_like(B_main)
    mg.mgdwf_solve(h, B_main, X, nrhs=12, tol=1e-10, max_outer=400, restart=8)  # warm-up: workspaces
    X.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = mg.mgdwf_solve(h, B_main, X, nrhs=12, tol=1e-10, max_outer=400, restart=8)
    torch.cuda.synchronize()
    s12 = (time.perf_counter() - t) / 12
    del X
    mg.mgdwf_set_mg_params(h, sq_params(mg, "f64", "f64"))
    x1 = torch.zeros_like(B_main[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    r64 = mg.mgdwf_solve(h, B_main[0].contiguous(), x1, nrhs=1, tol=1e-10, max_outer=400, restart=8)[0]
    torch.cuda.synchronize()
    s64 = time.perf_counter() - t
    del x1
    three = three_level_leg(mg, h, B_main, log)
    h.close()
    torch.cuda.empty_cache()
    r0 = reps[0]
    out = {"nvec": SQ_NVEC, "coarse_dof_per_site": 2 * SQ_NVEC, "sweep0_iters": SQ_SWEEP0, "nu": [SQ_NU, SQ_NU],
           "coarse_tol": SQ_CTOL, "setup_s": setup_s, "null_residual": srep["null_residual"],
           "mixed_12rhs_s_per_rhs": s12, "mixed_outer_iters": r0["outer_iters"],
           "mixed_fine_applies_per_rhs": r0["fine_applies"], "mixed_coarse_applies_per_rhs": r0["coarse_applies"],
           "mixed_max_true_relres": max(r["true_relres"] for r in reps),
           "mixed_phases_s": r0["phase_seconds"],
           "fp64_s_per_rhs": s64, "fp64_outer_iters": r64["outer_iters"], "fp64_fine_applies": r64["fine_applies"],
           "note": "coarse operator P^+ D^+D P (33-point stencil), FP32 coarse level, coarse solve as launched kernels",
           "three_level": three}
    log(f"squared-operator multigrid {out}")
    return out


L2_BLOCK, L2_NVEC, L2_NULL, L2_NU, L2_CTOL, L2_CMAX = (2, 2, 2, 2), 16, 50, 2, 0.1, 100


def three_level_leg(mg, h, B_main, log):
    """A third level under the squared multigrid of the squared leg (paper
    Sec. 2, recursion): 16 near-null vectors of A_c (50 CG steps from random
    coarse starts, seed 22), level-2 blocks of 2^4 coarse sites (a 2x2x2x4
    level-2 lattice, 32 dof per site), 2 + 2 MR steps on A_c, CG on A_cc to 0.1;
    the squared V-cycle's coarse solve (CG on A_c to 0.3) becomes one (V) or
    two (W) level-2 cycles.  12-RHS mixed-precision steps, FP32 levels."""
    import torch

    from inputs import random_coarse_starts

    Lc = tuple(L_MAIN[m] // BLOCK[m] for m in range(4))
    W0 = torch.from_numpy(random_coarse_starts(Lc, SQ_NVEC, L2_NVEC, 22)).cuda()
    out = {"block": L2_BLOCK, "nvec": L2_NVEC, "null_iters": L2_NULL, "nu": L2_NU, "coarse_tol": L2_CTOL,
           "coarse_maxiter": L2_CMAX}
    torch.cuda.synchronize()
    t = time.perf_counter()
    out["null_residual"] = mg.mgdwf_setup_level2(
        h, mg.make_level2_params(L2_BLOCK, L2_NVEC, L2_NULL, L2_NU, L2_CTOL, L2_CMAX, gamma=1), W0)
    torch.cuda.synchronize()
    out["setup_s"] = time.perf_counter() - t
    del W0
    mg.mgdwf_set_mg_params(h, sq_params(mg, "f32", "f32"))
    for gamma, name in ((1, "v_cycle"), (2, "w_cycle")):
        mg.mgdwf_set_level2_params(h, mg.make_level2_params(L2_BLOCK, L2_NVEC, L2_NULL, L2_NU, L2_CTOL, L2_CMAX,
                                                            gamma=gamma))
        X = torch.zeros_like(B_main)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = mg.mgdwf_solve(h, B_main, X, nrhs=12, tol=1e-10, max_outer=400, restart=8, allow_not_converged=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        del X
        r0 = reps[0]
        out[name] = {"s_per_rhs": el / 12, "outer_iters": r0["outer_iters"], "fine_applies_per_rhs": r0["fine_applies"],
                     "coarse_applies_per_rhs": r0["coarse_applies"], "coarse_phase_s": r0["phase_seconds"][1],
                     "max_true_relres": max(r["true_relres"] for r in reps)}
        log(f"three-level {name}: {out[name]}")
    mg.mgdwf_set_level2_params(h, mg.make_level2_params(L2_BLOCK, L2_NVEC, L2_NULL, L2_NU, L2_CTOL, L2_CMAX,
                                                        gamma=0))
    return out


def low_modes_leg(mg, log):
    """Low modes and the coarse space (paper Sec. 2, Fig. 1 right) on the
    small shape: 4^4 x Ls=8, m_f = 0.01, eps = 0.3 links, 2^4 blocks.  The
    lowest 24 eigenpairs of D^+D by 60 Lanczos steps on (D^+D)^-1 (each two
    FP64 squared-operator multigrid solves to 1e-12), and the fraction |P R e|^2 / |e|^2 of
    each inside three coarse spaces of 32 dof per block: the 9-point setup's
    (8 adaptive vectors and their reflections), the squared setup's (16
    adaptive vectors) and the one cut from the lowest 16 modes."""
    import numpy as np
    import torch

    from inputs import gaussian_fermion, prepare_gauge, random_starts

    Lq, Lsq, mfq, blk = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    NLM = 24
    t0 = time.perf_counter()
    U = torch.from_numpy(prepare_gauge(Lq, 0.3, 11)).cuda()
    kw = dict(sweeps=1, sweep0_iters=100, nu_pre=4, nu_post=4, coarse_tol=0.1, coarse_maxiter=200,
              fine_prec="f64", coarse_prec="f64")
    h9 = mg.Handle(Lq, Lsq, M5, mfq)
    mg.mgdwf_set_gauge(h9, U)
    mg.mgdwf_setup(h9, mg.make_mg_params(blk, 16, **kw), torch.from_numpy(random_starts(Lq, Lsq, 8, 21)).cuda())
    hs = mg.Handle(Lq, Lsq, M5, mfq)
    mg.mgdwf_set_gauge(hs, U)
    mg.mgdwf_setup(hs, mg.make_mg_params(blk, 16, squared=True, **kw),
                   torch.from_numpy(random_starts(Lq, Lsq, 16, 21)).cuda())
    t = time.perf_counter()
    ev, E, res = mg.mgdwf_low_modes(hs, torch.from_numpy(gaussian_fermion(Lq, Lsq, 31)).cuda(), NLM, 60,
                                    solve_tol=1e-12)
    lanczos_s = time.perf_counter() - t
    cov = {"nine_point_setup": mg.mgdwf_coarse_coverage(h9, E, NLM),
           "squared_setup": mg.mgdwf_coarse_coverage(hs, E, NLM)}
    mg.mgdwf_set_nullvecs(hs, blk, E[:16].contiguous(), 16)
    cov["lowest_16_modes"] = mg.mgdwf_coarse_coverage(hs, E, NLM)
    h9.close()
    hs.close()
    # the near-zero modes end at the largest relative gap of the spectrum
    lam = np.array(ev)
    k = int(np.argmax(lam[1:] / lam[:-1])) + 1
    out = {"lattice": "4^4 x Ls=8, m_f=0.01, eps=0.3, 2^4 blocks", "lanczos_steps": 60, "lanczos_s": lanczos_s,
           "eigenvalues": ev, "max_eig_residual": max(res), "near_zero_modes": k,
           "coverage": {kk: [round(x, 6) for x in v] for kk, v in cov.items()},
           "summary": {kk: {"near_zero_min": float(np.min(v[:k])), "near_zero_mean": float(np.mean(v[:k])),
                            "rest_mean": float(np.mean(v[k:])), "modes_0_15_min": float(np.min(v[:16]))}
                       for kk, v in cov.items()},
           "seconds": time.perf_counter() - t0}
    log(f"low modes: lambda {ev[0]:.3e} .. {ev[-1]:.3e}, residual {max(res):.1e}, summary {out['summary']}")
    return out


def mass_leg(mg, U_dev, B_main, log):
    """Iteration count versus quark mass (m_f = 0.01, 0.003, 0.001) on the main
    gauge field (eps = 0.3) and on a rougher one (eps = 0.6, seed 13), both with
    two APE steps: a fresh adaptive setup per mass, one point source,
    mixed-precision MG and, for the paper's comparison, CG on the normal
    equations (FP64), each to |b - D x| / |b| < 1e-10."""
    import torch

    from inputs import prepare_gauge, random_starts

    out = []
    U06 = None
    for eps in (0.3, 0.6):
        if eps == 0.6:
            U06 = torch.from_numpy(prepare_gauge(L_MAIN, 0.6, 13, ape_steps=2)).cuda()
        for mf in (0.01, 0.003, 0.001):
            h = mg.Handle(L_MAIN, LS, M5, mf)
            mg.mgdwf_set_gauge(h, U_dev if eps == 0.3 else U06)
            srep = mg.mgdwf_setup(h, mg_params(mg, "f64", "f64"),
                                  torch.from_numpy(random_starts(L_MAIN, LS, NVEC // 2, 21)).cuda())
            mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "f16"))
            b = B_main[0].contiguous()
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = mg.mgdwf_solve(h, b, x, nrhs=1, tol=1e-10, max_outer=400, restart=8, allow_not_converged=True)[0]
            torch.cuda.synchronize()
            mg_s = time.perf_counter() - t
            x.zero_()
            t = time.perf_counter()
            c = mg.mgdwf_cgne(h, b, x, tol=1e-10, max_iter=200000)
            torch.cuda.synchronize()
            cg_s = time.perf_counter() - t
            row = {"eps": eps, "m_f": mf, "null_residual": srep["null_residual"][-1],
                   "mg_outer_iters": r["outer_iters"], "mg_true_relres": r["true_relres"],
                   "mg_fine_applies": r["fine_applies"], "mg_s": mg_s, "cgne_iters": c["outer_iters"],
                   "cgne_fine_applies": c["fine_applies"], "cgne_s": cg_s}
            # the squared-operator multigrid (the paper's) on the same field, mass and source
            h.close()
            h = mg.Handle(L_MAIN, LS, M5, mf)
            mg.mgdwf_set_gauge(h, U_dev if eps == 0.3 else U06)
            mg.mgdwf_setup(h, sq_params(mg, "f64", "f64"),
                           torch.from_numpy(random_starts(L_MAIN, LS, SQ_NVEC, 21)).cuda())
            mg.mgdwf_set_mg_params(h, sq_params(mg, "f32", "f32"))
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rs = mg.mgdwf_solve(h, b, x, nrhs=1, tol=1e-10, max_outer=400, restart=8, allow_not_converged=True)[0]
            torch.cuda.synchronize()
            row.update({"sq_mg_outer_iters": rs["outer_iters"], "sq_mg_fine_applies": rs["fine_applies"],
                        "sq_mg_true_relres": rs["true_relres"], "sq_mg_s": time.perf_counter() - t,
                        "cgne_over_sq_mg_fine_applies": c["fine_applies"] / rs["fine_applies"]})
            log(f"mass scan {row}")
            out.append(row)
            h.close()
            del x
    return out


L_U1, LS_U1, BETA_U1, SEED_U1, M5_U1 = (20, 20), 8, 4.0, 7, 1.0


def u1_2d_leg(mg, log):
    """The paper's 2D U(1) test (Sec. 3, Fig. 2): 20^2 x 8, a quenched U(1)
    field (Wilson action, beta = 4, Metropolis, seed 7), 16 near-null vectors,
    blocks 4^2 x 8, m_f = 0.01 .. 0.10.  Per mass: the squared-operator
    multigrid (setup: CG on D^+D v = 0, 100 iterations; V-cycle: 4 + 4 MR
    steps, coarse CG to 0.1) preconditioning flexible GCR, against CG on the
    normal equations, both in FP64 on the two spin point sources lifted to the
    walls, to |b - D x| / |b| < 1e-10.  Cost in applications of the squared
    fine operator D^+D (half the D and D^+ applications), and the coarse
    operator applications per V-cycle (the coarse level's critical slowing,
    Fig. 2 right)."""
    import torch

    from inputs import point_sources2d, quenched_u1_2d, random_starts2d

    U = torch.from_numpy(quenched_u1_2d(L_U1, BETA_U1, SEED_U1)).cuda()
    b = torch.from_numpy(point_sources2d(L_U1, LS_U1)).cuda()
    starts = torch.from_numpy(random_starts2d(L_U1, LS_U1, 16, 21)).cuda()
    rows = []
    for k in range(1, 11):
        mf = 0.01 * k
        h = mg.Handle2D(L_U1, LS_U1, M5_U1, mf)
        mg.mgdwf_set_gauge(h, U)
        p = mg.make_mg_params((4, 4, 1, 1), 16, sweeps=1, sweep0_iters=100, nu_pre=4, nu_post=4, coarse_tol=0.1,
                              coarse_maxiter=500, fine_prec="f64", coarse_prec="f64", squared=True)
        t = time.perf_counter()
        srep = mg.mgdwf_setup(h, p, starts)
        setup_s = time.perf_counter() - t
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = mg.mgdwf_solve(h, b, x, nrhs=2, tol=1e-10, max_outer=300, restart=8, allow_not_converged=True)
        torch.cuda.synchronize()
        mg_s = time.perf_counter() - t
        cg_iters, cg_applies, cg_s = [], [], 0.0
        for r_ in range(2):
            y = torch.zeros_like(b[r_])
            t = time.perf_counter()
            c = mg.mgdwf_cgne(h, b[r_].contiguous(), y, tol=1e-10, max_iter=200000)
            torch.cuda.synchronize()
            cg_s += time.perf_counter() - t
            cg_iters.append(c["outer_iters"])
            cg_applies.append(c["fine_applies"])
        outer = r[0]["outer_iters"]
        row = {"m_f": round(mf, 2), "null_residual": srep["null_residual"][0], "setup_s": setup_s,
               "mg_outer_iters": outer, "mg_squared_applies_per_rhs": r[0]["fine_applies"] / 2.0,
               "mg_coarse_applies_per_vcycle": r[0]["coarse_applies"] / max(outer, 1),
               "mg_true_relres": max(q["true_relres"] for q in r), "mg_s_2rhs": mg_s,
               "cg_iters": cg_iters, "cg_squared_applies_per_rhs": sum(cg_applies) / 4.0, "cg_s_2rhs": cg_s}
        row["cg_over_mg_squared_applies"] = row["cg_squared_applies_per_rhs"] / row["mg_squared_applies_per_rhs"]
        log(f"2D U(1) {row}")
        rows.append(row)
        h.close()
    return {"lattice": "20^2 x 8", "beta": BETA_U1, "seed": SEED_U1, "M5": M5_U1, "nvec": 16, "block": [4, 4],
            "rows": rows}


N_TRAIN, N_EVAL = 200, 8


L_C5 = (24, 24, 24, 48)


def c5_field():
    """The learned leg's inference lattice 24^3 x 48 (eps 0.3, seed 16, 2 APE steps)."""
    from inputs import prepare_gauge
    return prepare_gauge(L_C5, 0.3, 16, ape_steps=2)


def training_fields():
    """The learned leg's 8^4 x 8 lattices (eps ~ U[0.2, 0.6] from seed 999,
    seeds 1000+i, 2 APE steps); generated on the host while the GPU runs the
    rest of the bench."""
    import numpy as np

    from inputs import prepare_gauge

    rng = np.random.default_rng(999)
    eps = 0.2 + 0.4 * rng.random(N_TRAIN + N_EVAL)
    return [prepare_gauge((8, 8, 8, 8), float(eps[i]), 1000 + i, ape_steps=2) for i in range(N_TRAIN + N_EVAL)]


def learned_leg(mg, h_main, fields_future, c5_future, log):
    """Learned near-null proposals: train the gauge-covariant network on the
    adaptive-setup bases of 200 seeded 8^4 x 8 lattices (eps ~ U[0.2, 0.6], 2
    APE; each lattice's full setup, then 20 Adam steps on it, streaming),
    then on the inference lattice 24^3 x 48 x 16 (eps 0.3, seed 16, 2 APE,
    m_f = 0.001) compare (a) the full setup (400 CG iterations from random
    starts), (b) the network's proposals + a 100-iteration refinement,
    (c) random starts + the same 100 iterations, each followed by a
    mixed-precision solve of one point source; the full setup is the fallback
    when (b)'s null residual exceeds twice (c)'s or its solve needs 25 % more
    outer iterations than (a)'s."""
    import torch

    from paper_1205_2933_amd import learned as ln

    t0 = time.perf_counter()
    fields = fields_future.result()
    gauge_wait_s = time.perf_counter() - t0
    n_train, n_eval = N_TRAIN, N_EVAL

    def make_handle(i):
        h = mg.Handle((8, 8, 8, 8), 8, M5, MF)
        mg.mgdwf_set_gauge(h, torch.from_numpy(fields[i]).cuda())
        return h

    held_out = []
    for i in range(n_train, n_train + n_eval):
        h = make_handle(i)
        ln.targets(h, mg_params(mg, "f64", "f64"), 2000 + i)
        held_out.append(h)
    net = mg.Net((8, 32, 32, 32, 2 * NVEC), lam=1.0, seed=3)
    loss0 = ln.evaluate(net, held_out)
    t = time.perf_counter()
    ln.train_stream(net, make_handle, n_train, mg_params(mg, "f64", "f64"), 20, 5e-3, 2e-4, seed=5, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    loss1 = ln.evaluate(net, held_out)
    for h in held_out:
        h.close()
    del fields
    log(f"trained: held-out loss {loss0:.4f} -> {loss1:.4f} in {train_s:.1f} s")

    out = {"train_lattices": f"{n_train} x 8^4x8, eps ~ U[0.2, 0.6] (seed 999), 2 APE; 20 Adam steps each",
           "train_steps": 20 * n_train, "train_s_incl_target_setups": train_s, "gauge_wait_s": gauge_wait_s,
           "held_out_loss_before": loss0, "held_out_loss_after": loss1,
           "inference_lattice": "24^3x48x16, eps 0.3 (seed 16), 2 APE, m_f 0.001"}
    mg.mgdwf_trim(h_main)
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    Uc5 = torch.from_numpy(c5_future.result()).cuda()
    out["c5_gauge_wait_s"] = time.perf_counter() - t0
    # each setup below gets a handle of its own, closed after its solve: one
    # handle holding one setup's basis (about 100 GB here) at a time
    def fresh():
        hh = mg.Handle(L_C5, LS, M5, MF)
        mg.mgdwf_set_gauge(hh, Uc5)
        return hh

    h = fresh()
    # one point source (spin 0, colour 0 at the origin, on the wall s = Ls - 1)
    b = torch.zeros(h.nfine, dtype=torch.complex128, device="cuda")
    b[(LS - 1) * 12] = 1.0

    def solve_iters(h):
        mg.mgdwf_trim(h)  # the setup's workspaces go first
        mem("learned leg, before a 24^3x48 solve")
        mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "f16"))
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = mg.mgdwf_solve(h, b, x, nrhs=1, tol=1e-10, max_outer=400, restart=8, allow_not_converged=True)[0]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        del x
        mg.mgdwf_trim(h)
        torch.cuda.empty_cache()
        mem("learned leg, after a 24^3x48 solve")
        return r["outer_iters"], r["true_relres"] < 1e-10, el

    short = mg.make_mg_params(BLOCK, NVEC, sweeps=1, sweep0_iters=100, sweep_iters=4, nu_pre=12, nu_post=12,
                              coarse_tol=0.1, coarse_maxiter=400, fine_prec="f64", coarse_prec="f64",
                              sweep0_check=SWEEP0_CHECK)
    # (a) the full setup from random starts
    torch.cuda.synchronize()
    t = time.perf_counter()
    rep = ln.targets(h, mg_params(mg, "f64", "f64"), 12)
    torch.cuda.synchronize()
    full_s = time.perf_counter() - t
    it_full, conv, s_full = solve_iters(h)
    h.close()
    torch.cuda.empty_cache()
    out["full_setup"] = {"sweep0_iters": 400, "setup_s": full_s, "null_residual": rep["null_residual"][-1],
                         "mg_iters": it_full, "converged": conv, "solve_s": s_full}
    # (c) the same short sweep from random starts: the reference of the fallback check
    h = fresh()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rep = mg.mgdwf_setup(h, short, ln.random_starts(h, NVEC // 2, 21))
    torch.cuda.synchronize()
    st = time.perf_counter() - t
    it, conv, s_r = solve_iters(h)
    h.close()
    torch.cuda.empty_cache()
    ref_null = rep["null_residual"][-1]
    out["random_short_setup"] = {"sweep0_iters": 100, "setup_s": st, "null_residual": ref_null,
                                 "mg_iters": it, "converged": conv, "solve_s": s_r}
    # (b) the network's proposals and the same short sweep, with the fallback
    h = fresh()
    r = ln.learned_setup(net, h, short, mg_params(mg, "f64", "f64"), seed=11, reference_null=ref_null)
    it, conv, s_l = solve_iters(h)
    fb = r["fallback"]
    if not fb and ln.needs_fallback(it, it_full):
        t = time.perf_counter()
        ln.targets(h, mg_params(mg, "f64", "f64"), 12)
        torch.cuda.synchronize()
        r["setup_s"] += time.perf_counter() - t
        fb = True
        it, conv, s_l = solve_iters(h)
    out["learned_setup"] = {"sweep0_iters": 100, "setup_s": r["setup_s"], "null_residual": r["null_residual"],
                            "fallback": fb, "mg_iters": it, "converged": conv, "solve_s": s_l,
                            "setup_speedup_vs_full": full_s / r["setup_s"]}
    # inference alone: the network's 12 proposals on the 24^3 x 48 x 16 lattice
    ln.propose(net, h, 1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    V = ln.propose(net, h, 2)
    torch.cuda.synchronize()
    out["inference_24c48_s"] = time.perf_counter() - t
    del V, Uc5
    h.close()
    torch.cuda.empty_cache()
    log(f"learned {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-solves", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ragged", action="store_true", help="skip the 48-solve ragged batch")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-setup comparison")
    ap.add_argument("--no-mass-scan", action="store_true", help="skip the iteration count versus m_f")
    ap.add_argument("--no-squared", action="store_true", help="skip the squared-operator multigrid step")
    ap.add_argument("--no-low-modes", action="store_true", help="skip the low-mode coverage on the 4^4 lattice")
    ap.add_argument("--no-u1", action="store_true", help="skip the 2D U(1) test problem")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1205_2933_amd as mg
    from inputs import point_sources, prepare_gauge, random_starts
    log("imports done")

    fields_future = c5_future = None
    if not args.no_learned:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(2)
        fields_future = pool.submit(training_fields)
        c5_future = pool.submit(c5_field)

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    U = prepare_main_gauge()
    log(f"inputs ready ({time.perf_counter() - t0:.1f} s)")
    h = mg.Handle(L, LS, M5, MF)
    U_dev = torch.from_numpy(U).to(dev)
    mg.mgdwf_set_gauge(h, U_dev)
    V0 = torch.from_numpy(random_starts(L, LS, NVEC // 2, 21)).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    srep = mg.mgdwf_setup(h, mg_params(mg, "f64", "f64"), V0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    del V0
    log(f"setup {setup_s:.2f} s, null residual {srep['null_residual']}")
    mem("after setup")

    nrhs = 12
    B = torch.from_numpy(point_sources(L, LS)).to(dev)
    X = torch.zeros_like(B)

    # ---- mixed precision, 12 right-hand sides per step; the FP32 Dslash
    # tiling is autotuned for 12 RHS first (part of the setup, not timed)
    tune = mg.mgdwf_tune(h, nrhs=nrhs, iters=10)
    tiling = {"id": tune["id"][tune["chosen"]], "tile": tune["tile"][tune["chosen"]],
              "coarse_mfma": {0: "16x16x16", 1: "16x16x32"}.get(tune["coarse_chosen"]),
              "coarse_us": tune["coarse_us"],
              "flags": tune["flags"][tune["chosen"]],
              "us": tune["us"][tune["chosen"]], "tilings_timed": len(tune["id"])}
    log(f"dslash tiling {tiling}")
    mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "f16"))

    def step():
        X.zero_()
        return mg.mgdwf_solve(h, B, X, nrhs=nrhs, tol=1e-10, max_outer=400, restart=8)

    for i in range(args.warmup):
        step()
        log(f"warmup step {i} done")
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = None
    for i in range(args.steps):
        reps = step()
        log(f"timed step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    mem("after the timed steps")
    ms_per_step = 1e3 * elapsed / args.steps
    worst = max(r["true_relres"] for r in reps)
    assert worst < 1e-10, worst
    s_per_rhs = elapsed / args.steps / nrhs
    x_check, b_check = X[0].cpu().numpy(), B[0].cpu().numpy()

    # ---- the same step with the D_c stored in BF16 (the other 16-bit format)
    mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "bf16"))
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps_bf = step()
    torch.cuda.synchronize()
    bf16_leg = {"s_per_rhs": (time.perf_counter() - t) / nrhs, "outer_iters": reps_bf[0]["outer_iters"],
                "max_true_relres": max(r["true_relres"] for r in reps_bf)}
    log(f"bf16 D_c step {bf16_leg}")

    # ---- the same step with the coarse CGNE as one persistent cooperative
    # kernel (one workgroup per CU, two coarse sites each) instead of graph replays
    mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "f16", coarse_graph="persistent"))
    step()  # warm: workspaces of the persistent path
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps_p = step()
    torch.cuda.synchronize()
    persistent_leg = {"s_per_rhs": (time.perf_counter() - t) / nrhs, "outer_iters": reps_p[0]["outer_iters"],
                      "coarse_solve_s": reps_p[0]["phase_seconds"][1],
                      "graph_path_coarse_solve_s": reps[0]["phase_seconds"][1],
                      "fallback": bool(reps_p[0]["flags"] & 8),
                      "max_true_relres": max(r["true_relres"] for r in reps_p)}
    log(f"persistent coarse step {persistent_leg}")
    mg.mgdwf_set_mg_params(h, mg_params(mg, "f32", "f16"))

    # ---- plain FP64 MG, single RHS, the same sources one after the other
    mg.mgdwf_set_mg_params(h, mg_params(mg, "f64", "f64"))
    fp64_times, fp64_iters = [], []
    for j in range(args.fp64_solves):
        x1 = torch.zeros_like(B[j % nrhs])
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = mg.mgdwf_solve(h, B[j % nrhs].contiguous(), x1, nrhs=1, tol=1e-10, max_outer=400, restart=8)[0]
        if j == 0:
            x1_first = x1.clone()
        torch.cuda.synchronize()
        fp64_times.append(time.perf_counter() - t)
        fp64_iters.append(r["outer_iters"])
        log(f"fp64 solve {j}: {fp64_times[-1]:.2f} s, {r['outer_iters']} iterations")

    # ---- error of each reduced-precision result against FP64 (the FP64 path
    # is the one parity-tested against the oracle at 1e-13)
    x0_mixed = torch.from_numpy(x_check).to(dev)  # the timed step's first solution
    g = torch.Generator(device=dev)
    g.manual_seed(77)
    psi = torch.randn(12 * int(np.prod(L)) * LS, dtype=torch.complex128, device=dev, generator=g)
    d64, d32 = torch.empty_like(psi), torch.empty_like(psi)
    mg.mgdwf_apply_dwf(h, psi, d64, prec="f64")
    mg.mgdwf_apply_dwf(h, psi, d32, prec="f32")
    Lc = tuple(L[m] // BLOCK[m] for m in range(4))
    cvec = torch.randn(Lc[::-1] + (2, NVEC), dtype=torch.complex128, device=dev, generator=g)
    c64 = torch.empty_like(cvec)
    mg.mgdwf_apply_coarse(h, cvec, c64, prec="f64")
    coarse_err = {}
    for cp in ("f32", "f16", "bf16"):
        cy = torch.empty_like(cvec)
        mg.mgdwf_apply_coarse(h, cvec, cy, prec=cp)
        coarse_err[cp] = float(torch.linalg.norm(cy - c64) / torch.linalg.norm(c64))
    precision = {
        "dslash_f32_relerr": float(torch.linalg.norm(d32 - d64) / torch.linalg.norm(d64)),
        "coarse_apply_relerr": coarse_err,
        "solution_mixed_vs_fp64_relerr": (float(torch.linalg.norm(x0_mixed - x1_first) / torch.linalg.norm(x1_first))
                                          if args.fp64_solves >= 1 else None),
        "note": "relative 2-norm differences from the FP64 path on the same input (random field, random coarse "
                "vector, and the first point source's solution)",
    }
    del psi, d64, d32, x0_mixed
    log(f"precision {precision}")

    # ---- Dslash bandwidth (HIP events on the library stream) and roofline
    V4 = int(np.prod(L))
    bytes64 = 2 * 12 * V4 * LS * 16 + 36 * V4 * 16
    ms64 = mg.mgdwf_time_kernel(h, mg.MGDWF_K_DSLASH, "f64", 1, 50)
    ms32 = mg.mgdwf_time_kernel(h, mg.MGDWF_K_DSLASH, "f32", 1, 50)
    gbs64 = bytes64 / (ms64 * 1e-3) / 1e9
    gbs32 = bytes64 / 2 / (ms32 * 1e-3) / 1e9
    # the launch the timed step makes: 12 right-hand sides in one FP32 Dslash
    bytes32_12 = nrhs * 2 * 12 * V4 * LS * 8 + 36 * V4 * 8
    ms32_12 = mg.mgdwf_time_kernel(h, mg.MGDWF_K_DSLASH, "f32", nrhs, 20)
    gbs32_12 = bytes32_12 / (ms32_12 * 1e-3) / 1e9
    msR = mg.mgdwf_time_kernel(h, mg.MGDWF_K_RESTRICT, "f32", 1, 10)
    msP = mg.mgdwf_time_kernel(h, mg.MGDWF_K_PROLONG, "f32", 1, 10)
    msC = mg.mgdwf_time_kernel(h, mg.MGDWF_K_COARSE, "f32", 1, 50)
    rp_bytes32 = (NVEC + 1) * 12 * V4 * LS * 8

    r0 = reps[0]
    counts = {"fine": int(r0["fine_applies"]), "vcycles": int(r0["outer_iters"]), "coarse": int(r0["coarse_applies"])}
    out = {
        "metric": "s to ||r||/||b||<1e-10, 16^3x32xLs16 m=0.001 (mixed+MRHS vs FP64); Dslash GB/s",
        "value": s_per_rhs,
        "unit": "s per RHS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fine level / f16 D_c on MFMA (f32 accumulate) / f64 outer GCR",
        "data": "synthetic",
        "config": {"workload": "DWF MG solve, 16^3x32 Ls=16 M5=1.8 m_f=0.001, SU(3) eps=0.3 + 2 APE, "
                               "12 point sources per step, blocks 4^4, Nv=24 (12 + reflections)",
                   "nrhs": nrhs, "tol": 1e-10},
        "rhs_per_s": 1.0 / s_per_rhs,
        "fp64_mg_s_per_rhs": float(np.sum(fp64_times)) / len(fp64_times),
        "fp64_mg_solves": len(fp64_times),
        "fp64_mg_outer_iters": fp64_iters,
        "mixed_over_fp64_speedup": float(np.sum(fp64_times)) / len(fp64_times) / s_per_rhs,
        "bf16_coarse_step": bf16_leg,
        "persistent_coarse_step": persistent_leg,
        "mixed_outer_iters": int(r0["outer_iters"]),
        "mixed_fine_applies_per_rhs": counts["fine"],
        "mixed_coarse_applies_per_rhs": counts["coarse"],
        "step_phases_s": {"presmooth_restrict": r0["phase_seconds"][0], "coarse_solve": r0["phase_seconds"][1],
                          "prolong_postsmooth": r0["phase_seconds"][2],
                          "outer_fgcr_and_fp64": r0["seconds"] - sum(r0["phase_seconds"]),
                          "note": "one timed step (12 RHS), V-cycle phases from HIP events on the solve's stream"},
        "max_true_relres": worst,
        "setup_s": setup_s,
        "null_residual": srep["null_residual"],
        "dslash": {"f64_us": ms64 * 1e3, "f64_GBs": gbs64, "f32_us": ms32 * 1e3, "f32_GBs": gbs32,
                   "f64_frac_peak": gbs64 / HBM_PEAK_GBS, "f32_frac_peak": gbs32 / HBM_PEAK_GBS,
                   "f32_12rhs_us": ms32_12 * 1e3, "f32_12rhs_GBs": gbs32_12},
        "restrict_f32_GBs": rp_bytes32 / (msR * 1e-3) / 1e9,
        "prolong_f32_GBs": rp_bytes32 / (msP * 1e-3) / 1e9,
        "coarse_apply_f32_us": msC * 1e3,
        "dslash_tiling": tiling,
        "precision": precision,
        "roofline": {"bound": "hbm", "kernel": dslash_kernel_name(tiling["flags"]) +
                     f", FP32, 12 RHS per launch, tiling {tiling['id']} {tiling['tile']}",
                     "achieved": gbs32_12, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs32_12 / HBM_PEAK_GBS,
                     "algorithmic_bytes": bytes32_12, "launch_us": ms32_12 * 1e3, "traffic": counted_traffic(tiling["id"])},
    }
    # the legs below change the main handle's setup, so they come last
    if not args.no_squared:
        mg.mgdwf_trim(h)
        torch.cuda.empty_cache()
        out["squared_operator_mg"] = squared_leg(mg, U_dev, B, log)
    if not args.no_low_modes:
        out["low_mode_coverage"] = low_modes_leg(mg, log)
    if not args.no_u1:
        out["u1_2d"] = u1_2d_leg(mg, log)
    if not args.no_mass_scan:
        mg.mgdwf_trim(h)
        torch.cuda.empty_cache()
        out["mass_scan"] = mass_leg(mg, U_dev, B, log)
    if not args.no_ragged:
        try:
            out["ragged_batch"] = ragged_leg(mg, h, B, log)
        except (mg.MgdwfError, AssertionError) as e:
            mem("ragged leg failed")
            out["ragged_batch"] = {"error": str(e)}
    if not args.no_learned:
        try:
            out["learned_setup"] = learned_leg(mg, h, fields_future, c5_future, log)
        except (mg.MgdwfError, AssertionError) as e:
            mem("learned leg failed")
            out["learned_setup"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(counts, x_check, b_check)
        log(f"oracle check of the GPU solution: {out['cpu_baseline']['oracle_check']}")
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
