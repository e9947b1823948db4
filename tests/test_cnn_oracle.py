"""Pins of the FP64 network reference: single-channel convolutions against
SciPy's correlate2d, every gradient against central finite differences, and
the closed form of Adam's first step."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


@pytest.mark.parametrize("d", [1, 2, 3])
def test_conv_matches_scipy_correlate2d(d):
    """A dilated 3x3 kernel is the (2d+1) x (2d+1) kernel with the taps d
    apart and zeros between them."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 9, 7))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    y = cnn.conv3x3(x, w, b, d)
    for co in range(2):
        ref = b[co]
        for ci in range(3):
            k = np.zeros((2 * d + 1, 2 * d + 1))
            k[::d, ::d] = w[co, ci]
            ref = ref + correlate2d(x[ci], k, mode="same", boundary="fill")
        assert np.allclose(y[co], ref, rtol=1e-13, atol=1e-13)


def _num_grad(f, a, h=1e-6):
    g = np.zeros_like(a)
    it = np.nditer(a, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = a[i]
        a[i] = old + h
        fp = f()
        a[i] = old - h
        fm = f()
        a[i] = old
        g[i] = (fp - fm) / (2 * h)
    return g


@pytest.mark.parametrize("channels,H,W,dil", [([2, 3, 3, 1], 5, 4, None), ([2, 4, 1], 3, 6, None),
                                              ([2, 3, 3, 1], 7, 8, [1, 3, 2])])
def test_gradients_match_finite_differences(channels, H, W, dil):
    rng = np.random.default_rng(1)
    params = [(w.copy(), rng.standard_normal(w.shape[0]) * 0.1) for w, _ in cnn.init_params(channels, 2)]
    x = rng.standard_normal((channels[0], H, W))
    t = rng.standard_normal((channels[-1], H, W))

    def loss():
        return cnn.mse(cnn.forward(params, x, dil)[-1], t)

    _, grads, dx = cnn.backward(params, cnn.forward(params, x, dil), t, dil)
    for (w, b), (gw, gb) in zip(params, grads):
        assert np.allclose(gw, _num_grad(loss, w), rtol=1e-6, atol=1e-9)
        assert np.allclose(gb, _num_grad(loss, b), rtol=1e-6, atol=1e-9)
    assert np.allclose(dx, _num_grad(loss, x), rtol=1e-6, atol=1e-9)


def test_batch_gradient_is_mean_of_samples():
    rng = np.random.default_rng(3)
    params = cnn.init_params([2, 3, 1], 4)
    xs = [rng.standard_normal((2, 4, 4)) for _ in range(3)]
    ts = [rng.standard_normal((1, 4, 4)) for _ in range(3)]
    loss, g = cnn.loss_and_grads_batch(params, xs, ts)
    singles = [cnn.backward(params, cnn.forward(params, x), t) for x, t in zip(xs, ts)]
    assert np.isclose(loss, np.mean([s[0] for s in singles]))
    assert np.allclose(g[0][0], np.mean([s[1][0][0] for s in singles], axis=0))


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(5)
    params = cnn.init_params([2, 3, 1], 6)
    grads = [(rng.standard_normal(w.shape), rng.standard_normal(b.shape)) for w, b in params]
    new, state = cnn.adam_step(params, grads, cnn.adam_init(params), lr=1e-3, eps=0.0)
    for (w, b), (nw, nb), (gw, gb) in zip(params, new, grads):
        assert np.allclose(nw - w, -1e-3 * np.sign(gw), rtol=1e-12, atol=1e-15)
        assert np.allclose(nb - b, -1e-3 * np.sign(gb), rtol=1e-12, atol=1e-15)
    assert state[0] == 1


def test_sample_round_trip_and_scale_invariance():
    rng = np.random.default_rng(5)
    H, W = 4, 6
    xp, r0, xn = (rng.standard_normal(H * W) for _ in range(3))
    unit = 3.0
    inp, tgt, s = cnn.make_sample(xp, r0, xn, H, W, unit)
    assert s == np.max(np.abs(r0))
    assert np.max(np.abs(inp[0])) == 1.0 and np.max(np.abs(inp[1])) == 1.0
    # the exact correction as network output reproduces the next solution
    np.testing.assert_allclose(cnn.apply_guess(xp, tgt, s, unit), xn, rtol=0, atol=1e-14)
    # inputs and targets do not depend on the units of the system
    inp2, tgt2, s2 = cnn.make_sample(8.0 * xp, 8.0 * r0, 8.0 * xn, H, W, unit)
    assert s2 == 8.0 * s
    np.testing.assert_array_equal(inp2, inp)
    np.testing.assert_array_equal(tgt2, tgt)
    # a zero residual: zero input channel and target, the guess is x_prev
    z_inp, z_tgt, z_s = cnn.make_sample(xp, np.zeros(H * W), xn, H, W, unit)
    assert z_s == 0.0 and not z_inp[0].any() and not z_tgt.any()
    np.testing.assert_array_equal(cnn.apply_guess(xp, np.ones(H * W), z_s, unit), xp)


def test_sample_target_solves_the_correction_equation(orc):
    """With r0 = b - A x_prev and x_next = A^-1 b, unit * A (s/unit target) = r0."""
    from paper_1604_06043_amd import inputs as I
    cd = I.config("c1", seed=0, n=8)
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    rng = np.random.default_rng(1)
    xp = rng.standard_normal(A.n)
    b = rng.standard_normal(A.n)
    xn = np.linalg.solve(A.dense(), b)
    r0 = b - orc.spmv(A, xp)
    unit = 7.0
    _, tgt, s = cnn.make_sample(xp, r0, xn, 8, 8, unit)
    np.testing.assert_allclose(A.dense() @ (tgt.ravel() * s / unit), r0, rtol=0, atol=1e-9 * np.abs(r0).max())
