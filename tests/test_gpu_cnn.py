"""Parity of the guess network's HIP kernels (through the C ABI) with the FP64
network reference in oracle/cnn.py.

Each kernel is checked on its own, fed the GPU's own BF16 tensors of the
previous step (so rounding from earlier layers does not blur the bar):

* sample preparation and the guess: bit-exact (divisions by the scales,
  rounding FP64 -> FP32 -> BF16 to nearest even, then x + (s / unit) out with
  each operation rounded);
* a convolution layer (forward, backward data): |gpu - ref| <= 2^-8 |ref| +
  3e-5 mag, where ref is the FP64 result from the same BF16 operands and mag
  the same sum over absolute values.  2^-8 is half a BF16 unit in the last
  place (the output is stored in BF16); 3e-5 >= (K-1) 2^-24 bounds FP32
  accumulation of K <= 288 products (exact in FP32);
* weight and bias gradients: |gpu - ref| <= 3e-5 mag (FP32 sums of at most a
  few hundred terms per thread and 256 workgroup partials);
* Adam: FP32 arithmetic, a few units in the last place of the parameter.

End to end, the BF16 network is also compared with the FP64 reference run
from the same input and BF16-rounded weights without intermediate rounding:
output within 2e-2 (relative norm); every gradient within 0.2 and at cosine
>= 0.98 of the FP64 one (reported: ReLU decisions flipped by rounding near
zero pass or block whole gradient values).
"""
import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu

CH = (2, 32, 32, 32, 32, 32, 1)
DIL = (1, 3, 9, 27, 3, 1)
HALF_ULP = 2.0 ** -8
ACC = 3e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def ms(torch_dev):
    from paper_1604_06043_amd import mstab
    mstab.load()
    return mstab


def bf16(a):
    """FP32 -> BF16 with round to nearest even, returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(vec):
    out, o = [], 0
    for cin, cout in zip(CH[:-1], CH[1:]):
        nw = cout * cin * 9
        w = np.asarray(vec[o:o + nw], np.float64).reshape(cout, cin, 3, 3)
        b = np.asarray(vec[o + nw:o + nw + cout], np.float64)
        out.append((w, b))
        o += nw + cout
    assert o == len(vec)
    return out


def make_params(seed, bias_scale=0.1):
    rng = np.random.default_rng(seed + 1000)
    ps = ocnn.init_params(CH, seed)
    return [(w, bias_scale * rng.standard_normal(b.shape)) for w, b in ps]


def gpu_params(params):
    """The parameters as the kernels use them: weights BF16(FP32(w)), biases FP32."""
    return [(bf16(np.float32(w)), np.float32(b).astype(np.float64)) for w, b in params]


def nhwc_to_chw(t, B, H, W, C):
    a = t.float().cpu().numpy().astype(np.float64)
    return a.reshape(B, H, W, C).transpose(0, 3, 1, 2)


def check(name, gpu, ref, mag, half_ulp=True, acc=ACC):
    tol = (HALF_ULP * np.abs(ref) if half_ulp else 0.0) + acc * mag + 1e-30
    err = np.abs(gpu - ref)
    worst = float(np.max(err / tol))
    assert worst <= 1.0, f"{name}: error {float(err.max()):.3e}, worst ratio to bar {worst:.3f}"
    return worst


class Net:
    """A network handle with one prepared batch and its GPU tensors."""

    def __init__(self, torch, ms, H, W, B, seed, max_batch=None, scales=None, unit=3.0,
                 dil=(1,) * 6):
        self.torch, self.ms, self.H, self.W, self.B = torch, ms, H, W, B
        self.unit, self.dil = unit, list(dil)
        self.net = ms.Cnn(H, W, max_batch or B, unit, dil)
        self.params = make_params(seed)
        self.net.set_params(flatten(self.params).astype(np.float32))
        rng = np.random.default_rng(seed)
        n = H * W
        scales = scales or [10.0 ** (k % 5 - 2) for k in range(B)]
        self.xp = [scales[i] * rng.standard_normal(n) for i in range(B)]
        self.r0 = [1e-3 * scales[i] * rng.standard_normal(n) for i in range(B)]
        self.xn = [self.xp[i] + 0.1 * scales[i] * rng.standard_normal(n) for i in range(B)]
        dev = "cuda"
        self.inp = torch.empty((B, 2 * n), dtype=torch.bfloat16, device=dev)
        self.tgt = torch.empty((B, n), dtype=torch.float32, device=dev)
        self.s = []
        for i in range(B):
            xp_d = torch.tensor(self.xp[i], device=dev)
            r_d = torch.tensor(self.r0[i], device=dev)
            xn_d = torch.tensor(self.xn[i], device=dev)
            self.s.append(self.net.prepare(xp_d, r_d, xn_d, self.inp[i], self.tgt[i]))
        torch.cuda.synchronize()

    def act(self, l):
        """Input of layer l as (B, C, H, W) float64 (layer 0: the prepared input)."""
        t = self.torch
        if l == 0:
            return nhwc_to_chw(self.inp, self.B, self.H, self.W, 2)
        full = t.empty((self.net.max_batch, self.H * self.W * 32), dtype=t.bfloat16, device="cuda")
        self.net.tensor(self.ms.CNN_T_ACT, l, full)
        return nhwc_to_chw(full[:self.B], self.B, self.H, self.W, 32)

    def f32(self, which, layer=0):
        t = self.torch
        full = t.empty((self.net.max_batch, self.H * self.W), dtype=t.float32, device="cuda")
        self.net.tensor(which, layer, full)
        return full[:self.B].cpu().numpy().astype(np.float64).reshape(self.B, 1, self.H, self.W)

    def dz(self, l):
        t = self.torch
        full = t.empty((self.net.max_batch, self.H * self.W * 32), dtype=t.bfloat16, device="cuda")
        self.net.tensor(self.ms.CNN_T_DZ, l, full)
        return nhwc_to_chw(full[:self.B], self.B, self.H, self.W, 32)


def per_layer_forward(net, samples):
    gp = gpu_params(net.params)
    worst = 0.0
    for l in range(6):
        x = net.act(l)
        y = net.act(l + 1) if l < 5 else net.f32(net.ms.CNN_T_OUT)
        w, b = gp[l]
        d = net.dil[l]
        for i in samples:
            ref = ocnn.conv3x3(x[i], w, b, d)
            mag = ocnn.conv3x3(np.abs(x[i]), np.abs(w), np.abs(b), d)
            if l < 5:
                ref = np.maximum(ref, 0.0)
            worst = max(worst, check(f"forward layer {l} sample {i}", y[i], ref, mag, half_ulp=l < 5))
    return worst


def per_layer_backward(net, samples_data):
    gp = gpu_params(net.params)
    B, H, W = net.B, net.H, net.W
    out = net.f32(net.ms.CNN_T_OUT)
    tgt = net.tgt.cpu().numpy().astype(np.float64).reshape(B, 1, H, W)
    dout = net.f32(net.ms.CNN_T_DOUT)
    npix = B * H * W
    ref = 2.0 * (out - tgt) / npix
    np.testing.assert_allclose(dout, ref, rtol=4 * 2.0 ** -24, atol=1e-38)
    # input gradients, layer by layer from the GPU's own upstream gradient
    acts = {l: net.act(l) for l in range(6)}
    dzs = {l: net.dz(l) for l in range(5)}
    up = {5: dout, 4: dzs[4], 3: dzs[3], 2: dzs[2], 1: dzs[1]}
    for l in range(5, 0, -1):
        w, d = gp[l][0], net.dil[l]
        for i in samples_data:
            r = ocnn.conv3x3_input_grad(up[l][i], w, d) * (acts[l][i] > 0.0)
            m = ocnn.conv3x3_input_grad(np.abs(up[l][i]), np.abs(w), d)
            check(f"backward data into layer {l - 1} sample {i}", dzs[l - 1][i], r, m)
    # weight and bias gradients summed over the batch
    _, g = net.net.get_params()
    gg = unflatten(g)
    grads = {5: dout, **{l: dzs[l] for l in range(5)}}
    for l in range(6):
        d = net.dil[l]
        rw = sum(ocnn.conv3x3_weight_grad(acts[l][i], grads[l][i], d) for i in range(B))
        mw = sum(ocnn.conv3x3_weight_grad(np.abs(acts[l][i]), np.abs(grads[l][i]), d) for i in range(B))
        rb = sum(grads[l][i].sum(axis=(1, 2)) for i in range(B))
        mb = sum(np.abs(grads[l][i]).sum(axis=(1, 2)) for i in range(B))
        check(f"dW layer {l}", gg[l][0], rw, mw, half_ulp=False)
        check(f"db layer {l}", gg[l][1], rb, mb, half_ulp=False)
    return g


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("H,W,B", [(5, 96, 3), (1, 32, 1), (33, 64, 2)])
def test_prepare_bit_exact(torch_dev, ms, H, W, B):
    print(f"[cnn prepare H={H} W={W} B={B}]", flush=True)
    net = Net(torch_dev, ms, H, W, B, seed=H)
    inp = net.inp.float().cpu().numpy().astype(np.float64).reshape(B, H * W, 2)
    tgt = net.tgt.cpu().numpy()
    for i in range(B):
        r_in, r_t, s = ocnn.make_sample(net.xp[i], net.r0[i], net.xn[i], H, W, net.unit)
        assert net.s[i] == s
        np.testing.assert_array_equal(inp[i][:, 0], bf16(np.float32(r_in[0].ravel())))
        np.testing.assert_array_equal(inp[i][:, 1], bf16(np.float32(r_in[1].ravel())))
        np.testing.assert_array_equal(tgt[i], np.float32(r_t.ravel()))


@pytest.mark.parametrize("H,W,B,max_batch,dil", [(5, 96, 3, 3, (1,) * 6), (7, 32, 2, 4, (1,) * 6),
                                                  (1, 64, 1, 1, (1,) * 6), (40, 96, 2, 2, DIL),
                                                  (5, 64, 2, 3, (2, 32, 5, 1, 7, 3))])
def test_forward_backward_per_layer(torch_dev, ms, H, W, B, max_batch, dil):
    print(f"[cnn layers H={H} W={W} B={B} max_batch={max_batch} dilation={dil}]", flush=True)
    net = Net(torch_dev, ms, H, W, B, seed=7 + H, max_batch=max_batch, dil=dil)
    loss = net.net.gradient(net.inp, net.tgt, B)
    per_layer_forward(net, range(B))
    g = per_layer_backward(net, range(B))
    out = net.f32(ms.CNN_T_OUT)
    tgt = net.tgt.cpu().numpy().astype(np.float64).reshape(out.shape)
    assert abs(loss - np.mean((out - tgt) ** 2)) <= 1e-6 * loss
    # the same batch again: identical gradient bits (fixed-order sums)
    loss2 = net.net.gradient(net.inp, net.tgt, B)
    _, g2 = net.net.get_params()
    assert loss2 == loss
    np.testing.assert_array_equal(g2, g)
    # forward alone gives the same output
    o = torch_dev.empty((B, H * W), dtype=torch_dev.float32, device="cuda")
    net.net.forward(net.inp, B, o)
    np.testing.assert_array_equal(o.cpu().numpy().reshape(out.shape), out.astype(np.float32))


def test_gradient_end_to_end_against_fp64(torch_dev, ms):
    print("[cnn end-to-end gradient]", flush=True)
    H, W, B = 30, 64, 2
    net = Net(torch_dev, ms, H, W, B, seed=3, dil=DIL)
    loss = net.net.gradient(net.inp, net.tgt, B)
    _, g = net.net.get_params()
    gg = unflatten(g)
    gp = gpu_params(net.params)
    x = net.act(0)
    tgt = net.tgt.cpu().numpy().astype(np.float64).reshape(B, 1, H, W)
    ref_loss, ref = ocnn.loss_and_grads_batch(gp, [x[i] for i in range(B)], [tgt[i] for i in range(B)],
                                              net.dil)
    print(f"  loss gpu {loss:.6e} fp64 {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    out = net.f32(ms.CNN_T_OUT)
    ref_out = np.stack([ocnn.forward(gp, x[i], net.dil)[-1] for i in range(B)])
    eo = np.linalg.norm(out - ref_out) / np.linalg.norm(ref_out)
    print(f"  output: relative error {eo:.2e}")
    worst_err, worst_cos = 0.0, 1.0
    for l in range(6):
        for name, a, r in (("dW", gg[l][0], ref[l][0]), ("db", gg[l][1], ref[l][1])):
            a, r = a.ravel(), r.ravel()
            e = np.linalg.norm(a - r) / np.linalg.norm(r)
            c = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
            print(f"  layer {l} {name}: relative error {e:.2e}, cosine {c:.5f}")
            worst_err, worst_cos = max(worst_err, e), min(worst_cos, c)
    # A pre-activation within rounding of zero can take the other ReLU branch
    # than in FP64; each such flip passes or blocks a whole gradient value, so
    # the gradient error grows like the square root of the flipped fraction
    # (a few tenths of a percent of the values: errors of several percent).
    # The gradients must still point the same way.
    assert eo <= 2e-2 and worst_err <= 0.2 and worst_cos >= 0.98


def test_adam_steps(torch_dev, ms):
    print("[cnn adam]", flush=True)
    H, W, B = 4, 32, 2
    net = Net(torch_dev, ms, H, W, B, seed=11)
    state = ocnn.adam_init(net.params)
    p_prev = flatten(net.params).astype(np.float32)
    for step in range(3):
        net.net.gradient(net.inp, net.tgt, B)
        _, g = net.net.get_params()
        net.net.adam_step(1e-3)
        p_gpu, _ = net.net.get_params()
        ref, state = ocnn.adam_step(unflatten(p_prev.astype(np.float64)),
                                    unflatten(g.astype(np.float64)), state, lr=1e-3)
        ref = flatten(ref)
        tol = 4 * 2.0 ** -24 * np.abs(ref) + 1e-3 * 1e-4
        err = np.abs(p_gpu - ref)
        assert np.all(err <= tol), f"step {step}: {err.max():.3e}"
        assert np.any(p_gpu != p_prev)
        p_prev = p_gpu


def test_guess_bit_exact_and_zero_residual(torch_dev, ms):
    print("[cnn guess]", flush=True)
    torch = torch_dev
    H, W = 6, 64
    net = Net(torch, ms, H, W, 1, seed=5)
    rng = np.random.default_rng(9)
    xp = rng.standard_normal(H * W)
    r0 = 3e-4 * rng.standard_normal(H * W)
    xp_d, r_d = torch.tensor(xp, device="cuda"), torch.tensor(r0, device="cuda")
    xg = torch.empty_like(xp_d)
    net.net.guess(xp_d, r_d, xg)
    out = net.f32(ms.CNN_T_OUT)[0].ravel()
    _, _, s = ocnn.make_sample(xp, r0, None, H, W, net.unit)
    np.testing.assert_array_equal(xg.cpu().numpy(), ocnn.apply_guess(xp, out, s, net.unit))
    # the network's output is that of the prepared input of this system
    inp = torch.empty((1, 2 * H * W), dtype=torch.bfloat16, device="cuda")
    net.net.prepare(xp_d, r_d, None, inp, None)
    o = torch.empty((1, H * W), dtype=torch.float32, device="cuda")
    net.net.forward(inp, 1, o)
    np.testing.assert_array_equal(o.cpu().numpy().ravel(), out.astype(np.float32))
    # in place (x_guess aliases x_prev)
    xg2 = xp_d.clone()
    net.net.guess(xg2, r_d, xg2)
    np.testing.assert_array_equal(xg2.cpu().numpy(), xg.cpu().numpy())
    # r0 = 0 (x_prev already solves the system): s = 0 and the guess is x_prev
    z = torch.zeros_like(r_d)
    assert net.net.prepare(xp_d, z, None, inp, None) == 0.0
    assert not inp.float().view(-1, 2)[:, 0].abs().sum().item()
    net.net.guess(xp_d, z, xg)
    np.testing.assert_array_equal(xg.cpu().numpy(), xp)


def test_residual_entry_point(torch_dev, ms, orc):
    """mstab_residual is b - A x with the bit-exact product kernel."""
    from paper_1604_06043_amd import inputs as I
    torch = torch_dev
    cd = I.config("c4", seed=0, n=64)
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    Ag = ms.mstab_assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt)
    solver = ms.Solver(Ag, 4, 2)
    rng = np.random.default_rng(2)
    x, b = rng.standard_normal(A.n), rng.standard_normal(A.n)
    r = torch.empty(A.n, dtype=torch.float64, device="cuda")
    t0, _ = solver.mv_count()
    n2 = solver.residual(torch.tensor(b, device="cuda"), torch.tensor(x, device="cuda"), r)
    ref = b - orc.spmv(A, x)
    np.testing.assert_array_equal(r.cpu().numpy(), ref)
    assert abs(n2 - ref @ ref) <= 1e-12 * (ref @ ref)
    assert solver.mv_count()[0] == t0 + 1
    solver.close()


def test_bad_arguments(torch_dev, ms):
    for H, W, mb, unit, dil in ((0, 32, 1, 1.0, None), (4, 0, 1, 1.0, None), (4, 48, 1, 1.0, None),
                                (4, 32, 0, 1.0, None), (4, 32, 1, 0.0, None),
                                (4, 32, 1, float("inf"), None), (4, 32, 1, 1.0, (1, 1, 0, 1, 1, 1)),
                                (4, 32, 1, 1.0, (1, 1, 33, 1, 1, 1))):
        with pytest.raises(ms.MstabError):
            ms.Cnn(H, W, mb, unit, dil)
    net = ms.Cnn(4, 32, 2)
    with pytest.raises(ms.MstabError):
        net.set_params(np.zeros(10, np.float32))
    inp = torch_dev.zeros((3, 256), dtype=torch_dev.bfloat16, device="cuda")
    with pytest.raises(ms.MstabError):
        net.forward(inp, 3)
    with pytest.raises(ms.MstabError):
        net.adam_step(0.0)


def test_full_size_512(torch_dev, ms):
    """The training launch configuration (512 x 512 grid, batch 8, the
    guess network's dilations): every kernel against the reference on the
    first and last sample."""
    print("[cnn full size 512x512 batch 8]", flush=True)
    H = W = 512
    B = 8
    net = Net(torch_dev, ms, H, W, B, seed=21, dil=DIL)
    net.net.gradient(net.inp, net.tgt, B)
    per_layer_forward(net, (0, B - 1))
    per_layer_backward(net, (0, B - 1))
