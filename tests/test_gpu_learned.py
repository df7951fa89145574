"""Learned local solve: GPU training kernels against the FP64 oracle network,
training progress, and what the trained network gains over the method
without a local solve on the interior subdomains."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from oracle.conv import ConvNet  # noqa: E402

pytestmark = pytest.mark.gpu
CH = [4, 32, 32, 32, 4]


def bf16(a):
    """Round-to-nearest-even to BF16 values (held in float32)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split(flat):
    W, b, o = [], [], 0
    for l in range(4):
        nw = CH[l + 1] * CH[l] * 27
        W.append(flat[o:o + nw].reshape(CH[l + 1], CH[l], 3, 3, 3).astype(np.float64))
        o += nw
        b.append(flat[o:o + CH[l + 1]].astype(np.float64))
        o += CH[l + 1]
    return W, b


def pressure_mask(g):
    """Velocity on every node; pressure on the Q1 nodes, i.e. odd grid
    positions of the Dirichlet local problem (its first node is odd in Q2
    coordinates)."""
    m = np.ones((4, g, g, g))
    odd = (np.arange(g) % 2 == 1)
    m[3] = np.einsum("i,j,k->ijk", odd, odd, odd)
    return m


@pytest.fixture(scope="module")
def solver16():
    print("[gpu] learned: setup 16^3", flush=True)
    s = G.Solver(16, 4)
    info = s.learned_init(seed=7)
    assert info.grid == 11 and info.subdomains == 8
    yield s
    s.close()


def test_gradients_match_fp64_oracle(solver16):
    """Loss and every gradient entry against the FP64 oracle network with the
    GPU's storage formats: the working weights (BF16 values), BF16 inputs and
    BF16 activations after every layer.  What is left is the GPU's FP32
    accumulation (and the odd activation that FP32 rounds to the other BF16
    neighbour), so each entry of dW and db must agree to 1e-4 of its layer's
    largest entry."""
    s = solver16
    g = s.learned.grid
    rng = np.random.default_rng(0)
    B = 2
    X = bf16(rng.standard_normal((B, 4, g, g, g)) * pressure_mask(g))
    T = rng.standard_normal((B, 4, g, g, g)).astype(np.float32)
    loss, grads = s.learned_loss_grad(X, T)
    Wf = s.learned_weights(which=1)
    assert np.array_equal(bf16(Wf), Wf)  # the working copy holds BF16 values
    W, b = split(Wf)
    net = ConvNet(CH, weights=(W, b))
    lo, gW, gb, _ = net.loss_and_grads(X.astype(np.float64), T.astype(np.float64), pressure_mask(g)[None],
                                       act_round=lambda a: bf16(a).astype(np.float64))
    Gg, Gb = split(grads)
    print(f"[gpu] loss gpu {loss:.6e} oracle {lo:.6e}", flush=True)
    assert abs(loss - lo) / lo < 1e-5
    for l in range(4):
        ew = np.abs(Gg[l] - gW[l]).max() / np.abs(gW[l]).max()
        eb = np.abs(Gb[l] - gb[l]).max() / max(np.abs(gb[l]).max(), 1e-30)
        print(f"[gpu] layer {l}: dW max entry err {ew:.2e}, db max entry err {eb:.2e} (of the layer's largest)",
              flush=True)
        assert ew < 1e-4 and eb < 1e-4


def test_training_and_ablation(solver16):
    s = solver16
    b = torch.zeros(s.n_free, dtype=torch.float64, device="cuda")
    s.rhs(b)

    def iterations(mode, tau=1e30):
        s.set_local_solver(mode, tau)
        x = torch.zeros_like(b)
        info = s.fgmres(b, x, rtol=1e-8, max_it=400, raise_on_noconv=False)[0]
        return info.iterations, info.true_rel_res

    it_lu, _ = iterations("lu")
    it_none, _ = iterations("none")
    it_untrained, _ = iterations("learned")
    hist = s.learned_train(solves=4, steps=600, batch=32, lr=2e-3, seed=3)
    first, last = float(np.mean(hist[:20])), float(np.mean(hist[-20:]))
    it_trained, rel = iterations("learned")
    it_fb, rel_fb = iterations("learned", tau=0.7)
    n_learned, n_fb = s.learned_stats()
    s.set_local_solver("lu")
    print(f"[gpu] loss {first:.3e} -> {last:.3e}; iterations: LU {it_lu}, none {it_none}, "
          f"untrained {it_untrained}, trained {it_trained}, trained+fallback {it_fb}; "
          f"learned solves {n_learned}, fallbacks {n_fb}", flush=True)
    assert last < 0.5 * first
    assert rel <= 1e-8 and rel_fb <= 1e-8
    assert it_trained < it_none and it_trained < it_untrained
    assert it_lu <= it_fb <= it_trained
