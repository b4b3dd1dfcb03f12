"""GPU parity of the near-null proposal network against the oracle.

The network, its lift to five dimensions (the free-field wall profile shared
by every low mode, paper Sec. 2 last paragraph) and the training loss against
a block basis (paper Sec. 1-2: P R projects onto the coarse space) are
computed by the library in FP32 with BF16 weights.  The oracle runs in FP64 on
the same BF16-rounded weights, so the only difference is FP32 rounding:
proposals within 1e-5, loss within 1e-5 and the weight gradient within 1e-4
(normwise, relative).
"""
import numpy as np
import pytest
import torch

from inputs import prepare_gauge, random_starts
from oracle import nullnet as nn
from oracle import transfer as ot

pytestmark = pytest.mark.gpu

M5 = 1.8

CASES = [
    # (L, Ls, block, nvec, channels)
    ((4, 4, 4, 4), 8, (2, 2, 2, 2), 8, (2, 8, 8, 8, 8)),
    ((6, 4, 2, 4), 6, (2, 2, 2, 2), 6, (3, 5, 7, 6, 12)),   # ragged channel counts, L_y = 2 (aliased +-y)
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def bf16_round(w32: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (nearest, ties to even), returned as float64."""
    b = w32.astype(np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def weights(channels, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    Ws = [(scale * rng.standard_normal((9, o, i)) / np.sqrt(9 * i)).astype(np.float32)
          for i, o in zip(channels[:-1], channels[1:])]
    flat = np.concatenate([w.ravel() for w in Ws])
    return flat, [bf16_round(w) for w in Ws]


def noise(C, L, seed):
    rng = np.random.default_rng(seed)
    shp = (C,) + tuple(L[::-1]) + (3,)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def make(case, mg, lam=1.0, wseed=5):
    L, Ls, block, nvec, ch = case
    U = prepare_gauge(L, 0.4, 31)
    h = mg.Handle(L, Ls, M5, 0.01)
    mg.mgdwf_set_gauge(h, dev(U))
    net = mg.Net(ch, lam)
    flat, Ws = weights(ch, wseed)
    assert net.nweights == flat.size
    mg.mgdwf_net_set_weights(net, torch.from_numpy(flat))
    eta = noise(ch[0], L, 7)
    return U, h, net, Ws, eta


@pytest.mark.parametrize("case", CASES)
def test_propose_matches_oracle(case, cuda):
    import paper_1205_2933_amd as mg
    L, Ls, block, nvec, ch = case
    U, h, net, Ws, eta = make(case, mg)
    nh = ch[4] // 4
    V = torch.empty(nh * h.nfine, dtype=torch.complex128, device="cuda")
    mg.mgdwf_net_propose(net, h, dev(eta), V)
    ref = nn.propose(eta, U, Ws, nh, Ls, M5)
    got = V.cpu().numpy().reshape(ref.shape)
    assert rel(got, ref) < 1e-5
    for k in range(nh):
        assert rel(got[k], ref[k]) < 1e-5


@pytest.mark.parametrize("case", CASES)
def test_weights_roundtrip(case, cuda):
    import paper_1205_2933_amd as mg
    flat, _ = weights(case[4], 5)
    _, h, net, _, _ = make(case, mg)
    assert np.array_equal(mg.mgdwf_net_get_weights(net).numpy(), flat)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_loss_and_gradient_match_oracle(case, lam, cuda):
    import paper_1205_2933_amd as mg
    L, Ls, block, nvec, ch = case
    U, h, net, Ws, eta = make(case, mg, lam)
    nh = ch[4] // 4
    V0 = random_starts(L, Ls, nvec, 41)
    mg.mgdwf_set_nullvecs(h, block, dev(V0), nvec)
    loss, g = mg.mgdwf_net_grad(net, h, dev(eta))

    Vhat = ot.build_basis(V0, block)
    out, cache = nn.forward(eta, U, Ws)
    f = nn.to_spinors(out, nh)
    L_ref, gf = nn.loss_and_grad(f, Vhat, block, Ls, M5, lam)
    dWs, _ = nn.backward(nn.from_spinors(gf), U, Ws, cache)
    g_ref = np.concatenate([d.ravel() for d in dWs])
    assert abs(loss - L_ref) < 1e-5 * abs(L_ref)
    assert rel(g.numpy(), g_ref) < 1e-4
    # every layer, not only the largest
    off = 0
    for d in dWs:
        assert rel(g.numpy()[off:off + d.size], d.ravel()) < 1e-4
        off += d.size


def test_grad_requires_basis(cuda):
    import paper_1205_2933_amd as mg
    _, h, net, _, eta = make(CASES[0], mg)
    with pytest.raises(mg.MgdwfError, match="STATE"):
        mg.mgdwf_net_grad(net, h, dev(eta))


def test_training_lowers_the_loss(cuda):
    """Adam steps on the loss; the loss reported by a step equals grad's loss."""
    import paper_1205_2933_amd as mg
    case = CASES[0]
    L, Ls, block, nvec, ch = case
    U, h, net, Ws, eta = make(case, mg)
    mg.mgdwf_set_nullvecs(h, block, dev(random_starts(L, Ls, nvec, 41)), nvec)
    e = dev(eta)
    l0, _ = mg.mgdwf_net_grad(net, h, e, want_grad=False)
    first = mg.mgdwf_net_train_step(net, h, e, 1e-2)
    assert first == l0
    losses = [mg.mgdwf_net_train_step(net, h, e, 1e-2) for _ in range(30)]
    # a random target space of 4 of 768 dimensions per block and chirality
    # leaves the first term near 1; the steps still have to lower it
    assert losses[-1] < l0 - 0.01
    assert all(np.isfinite(losses))


def test_library_training_loop_and_network_files(cuda, tmp_path):
    """mgdwf_net_train equals the same Adam steps taken one call at a time
    (constant learning rate: the same arithmetic, bit for bit); a saved
    network reloads its weights and Adam state, so training continues
    identically; other channel counts and foreign files are refused."""
    import paper_1205_2933_amd as mg
    case = CASES[0]
    L, Ls, block, nvec, ch = case
    U, h, net, Ws, eta = make(case, mg)
    mg.mgdwf_set_nullvecs(h, block, dev(random_starts(L, Ls, nvec, 41)), nvec)
    etas = [dev(noise(ch[0], L, 100 + k)) for k in range(6)]
    _, h2, net2, _, _ = make(case, mg)
    mg.mgdwf_set_nullvecs(h2, block, dev(random_starts(L, Ls, nvec, 42)), nvec)
    one = [mg.mgdwf_net_train_step(net, (h, h2)[k % 2], etas[k], 3e-3) for k in range(6)]
    loop = mg.mgdwf_net_train(net2, [h, h2], etas, 3e-3, 3e-3)
    assert one == loop
    assert torch.equal(mg.mgdwf_net_get_weights(net), mg.mgdwf_net_get_weights(net2))
    path = tmp_path / "net.bin"
    mg.mgdwf_net_save(net, path)
    net3 = mg.Net(ch, 1.0, seed=9)
    mg.mgdwf_net_load(net3, path)
    assert torch.equal(mg.mgdwf_net_get_weights(net3), mg.mgdwf_net_get_weights(net))
    a = mg.mgdwf_net_train(net, [h], etas[:3], 3e-3)
    b = mg.mgdwf_net_train(net3, [h], etas[:3], 3e-3)
    assert a == b
    assert torch.equal(mg.mgdwf_net_get_weights(net3), mg.mgdwf_net_get_weights(net))
    other = mg.Net((2, 8, 8, 4, 8), 1.0)
    with pytest.raises(mg.MgdwfError, match="STATE"):
        mg.mgdwf_net_load(other, path)
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a network" * 8)
    with pytest.raises(mg.MgdwfError, match="INVALID_ARG"):
        mg.mgdwf_net_load(net3, junk)
    for x in (h, h2):
        x.close()
