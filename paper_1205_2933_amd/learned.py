"""Training and use of the gauge-covariant near-null proposal network.

Orchestration of C-ABI calls only: the network's forward pass, loss,
backward pass and Adam step run in the library (mgdwf_net_*), and so do the
adaptive setups that produce the training targets and refine the proposals.

Workflow (the adaptive setup of the paper's Sec. 2 decides what is kept and is the
fallback):

1. ``targets``: on each training lattice, a full adaptive setup (mgdwf_setup)
   installs the block basis the network learns to reproduce.
2. ``train``: Adam steps, one training lattice and one fresh draw of the
   Gaussian input channels per step.
3. ``learned_setup``: on a new lattice the network proposes the Nv/2 start
   vectors, one short setup sweep refines them (mgdwf_setup with a small
   sweep-0 iteration count) and the coarse operator is built from the result.
   Fallback to the full adaptive setup from random starts: if the median null
   residual |D v|/|v| after the refinement is above twice that of the same
   short sweep from random starts (``reference_null``), or, once the first
   solve has run, if it took more than 25 % more outer iterations than the
   last full adaptive setup gave (``needs_fallback``).
"""

from __future__ import annotations

import time

import torch

from . import _lib as mg


def noise(channels: int, V4: int, seed: int, device: str = "cuda") -> torch.Tensor:
    """Seeded input channels: complex Gaussian [channels][x4][colour]."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(channels * V4 * 3, dtype=torch.complex128, device=device, generator=g)


def random_starts(h: mg.Handle, n: int, seed: int) -> torch.Tensor:
    """Seeded complex Gaussian start vectors for the adaptive setup."""
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    return torch.randn(n * h.nfine, dtype=torch.complex128, device="cuda", generator=g)


def targets(h: mg.Handle, params: mg.mgdwf_mg_params, seed: int) -> dict:
    """Full adaptive setup on h from random starts; the basis it installs on h
    is the training target for that lattice."""
    V0 = random_starts(h, params.nvec // 2, seed)
    rep = mg.mgdwf_setup(h, params, V0)
    del V0
    return rep


def _lr_at(lr: float, lr_final: float, k: int, total: int) -> float:
    return lr * (lr_final / lr) ** (k / max(1, total - 1))


def _train_span(net: mg.Net, handles, k0: int, k1: int, total: int, lr: float, lr_final: float, seed: int) -> list:
    """Steps k0 .. k1 - 1 of a geometric schedule over `total` steps, in one
    mgdwf_net_train call (step k on handles[k % len(handles)], input draw
    seed + k)."""
    n = len(handles)
    hs = [handles[(k0 + j) % n] for j in range(min(n, k1 - k0))]
    etas = [noise(net.channels[0], handles[k % n].V4, seed + k) for k in range(k0, k1)]
    return mg.mgdwf_net_train(net, hs, etas, _lr_at(lr, lr_final, k0, total), _lr_at(lr, lr_final, k1 - 1, total))


def train(net: mg.Net, handles, steps: int, lr: float, lr_final: float | None = None, seed: int = 0,
          log=None) -> list:
    """Adam steps cycling over the handles (each with its target basis
    installed); learning rate decays geometrically from lr to lr_final.  The
    steps run in the library (mgdwf_net_train), 100 per call."""
    losses = []
    lr_final = lr if lr_final is None else lr_final
    for k0 in range(0, steps, 100):
        k1 = min(steps, k0 + 100)
        losses += _train_span(net, handles, k0, k1, steps, lr, lr_final, seed)
        if log:
            log(f"train step {k1 - 1}: loss {losses[-1]:.4f}")
    return losses


def train_stream(net: mg.Net, make_handle, n_lattices: int, params: mg.mgdwf_mg_params, steps_per_lattice: int,
                 lr: float, lr_final: float | None = None, seed: int = 0, log=None) -> list:
    """Training that streams over lattices: for lattice i, make_handle(i)
    returns a handle with its gauge field set, a full adaptive setup installs
    the target basis, steps_per_lattice Adam steps run on it (one
    mgdwf_net_train call) and the handle is released.  The learning rate
    decays geometrically over all steps."""
    losses = []
    total = n_lattices * steps_per_lattice
    lr_final = lr if lr_final is None else lr_final
    for i in range(n_lattices):
        h = make_handle(i)
        targets(h, params, seed + 7919 * i + 1)
        k0 = i * steps_per_lattice
        losses += _train_span(net, [h], k0, k0 + steps_per_lattice, total, lr, lr_final, seed)
        h.close()
        if log and (i % 25 == 0 or i == n_lattices - 1):
            log(f"lattice {i}: loss {sum(losses[-steps_per_lattice:]) / steps_per_lattice:.4f}")
    return losses


def evaluate(net: mg.Net, handles, seed: int = 10 ** 6) -> float:
    """Mean training loss over the handles on fresh input draws."""
    tot = 0.0
    for i, h in enumerate(handles):
        loss, _ = mg.mgdwf_net_grad(net, h, noise(net.channels[0], h.V4, seed + i), want_grad=False)
        tot += loss
    return tot / len(handles)


def propose(net: mg.Net, h: mg.Handle, seed: int) -> torch.Tensor:
    """The network's Nv/2 lifted proposals on h's lattice (canonical complex128)."""
    V = torch.empty(net.nh * h.nfine, dtype=torch.complex128, device="cuda")
    mg.mgdwf_net_propose(net, h, noise(net.channels[0], h.V4, seed), V)
    return V


def needs_fallback(outer_iters: int, reference_iters: int, slack: float = 1.25) -> bool:
    """True if a solve after the learned setup took more than `slack` times the
    outer iterations of the last full adaptive setup."""
    return outer_iters > slack * reference_iters


def learned_setup(net: mg.Net, h: mg.Handle, params_short: mg.mgdwf_mg_params, params_full: mg.mgdwf_mg_params,
                  seed: int, reference_null: float | None = None, fallback_ratio: float = 2.0) -> dict:
    """Proposals + one short refinement sweep; the full setup if the refined
    vectors' null residual exceeds fallback_ratio x reference_null (the same
    short sweep from random starts)."""
    if params_short.nvec != 2 * net.nh:
        raise ValueError("the network proposes nvec/2 start vectors")
    torch.cuda.synchronize()
    t = time.perf_counter()
    V0 = propose(net, h, seed)
    rep = mg.mgdwf_setup(h, params_short, V0)
    del V0
    torch.cuda.synchronize()
    out = {"setup_s": time.perf_counter() - t, "null_residual": rep["null_residual"][-1], "fallback": False}
    if reference_null is not None and out["null_residual"] > fallback_ratio * reference_null:
        t = time.perf_counter()
        rep = targets(h, params_full, seed + 1)
        torch.cuda.synchronize()
        out.update(setup_s=out["setup_s"] + time.perf_counter() - t, null_residual=rep["null_residual"][-1],
                   fallback=True)
    return out
