"""The training script's network and sampler (paper_2203_11043_amd/closure_train.py)
agree with the closure oracle's definitions, so trained weights mean the same
thing to the trainer, the oracle and the GPU network."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import closure as C  # noqa: E402


@pytest.fixture(scope="module")
def T():
    from paper_2203_11043_amd import closure_train
    return closure_train


def test_layer_table_matches_oracle(T):
    assert [(n, ci, co) for n, ci, co, _ in T.LAYERS] == [(n, ci, co) for n, _, ci, co, _ in C.LAYERS]


def test_network_matches_oracle(T):
    rng = np.random.default_rng(1)
    w = rng.normal(0.0, 0.05, size=C.n_weights())
    model = T.UNet().double()
    k = 0
    for name, *_ in T.LAYERS:
        p = model.conv[name].weight
        m = p.numel()
        with torch.no_grad():
            p.copy_(torch.from_numpy(w[k:k + m].reshape(p.shape)))
        k += m
    assert np.array_equal(model.flat_weights(), w.astype(np.float32))
    rho = rng.uniform(0.0, 3.0, size=(C.NG, C.NG, C.NG))
    with torch.no_grad():
        got = model(torch.from_numpy(rho)[None, None])[0].numpy()
    want = C.network(rho, w)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-10 * np.abs(want).max())
    # bf16 mode rounds at the oracle's points
    model.quant = True
    with torch.no_grad():
        got_q = model(torch.from_numpy(rho)[None, None].float().double())[0].numpy()
    want_q = C.network(rho, w, quantize=C.bf16)
    assert np.max(np.abs(got_q - want_q)) <= 1e-2 * np.abs(want_q).max()


def test_sampler_matches_oracle(T):
    rng = np.random.default_rng(2)
    Fg = rng.normal(size=(3, C.NG, C.NG, C.NG))
    u = rng.uniform(1.0, C.NG - 2.0, size=(500, 3))
    got = T.catmull_rom_sample(torch.from_numpy(Fg)[None], torch.from_numpy(u)[None])[0].numpy()
    want = C.interpolate(Fg, u[:, 0], u[:, 1], u[:, 2], np.zeros(3), 1.0).T
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_coulomb_constant(T, orc):
    assert T.coulomb_K(11.7) == pytest.approx(orc.coulomb_constant(11.7), rel=1e-14)
