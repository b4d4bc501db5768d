"""Pins of the oracle's learned-preconditioner network (3x3x3 convolutions,
zero padding, ReLU) and its training step, against torch's CPU FP64 library
routines, finite differences and closed forms. No GPU."""
import numpy as np
import pytest
import torch

import synthetic


def _w(seed, cin, cout, scale=0.3):
    return (synthetic.uniform(seed, 27 * cin * cout) * scale).reshape(27, cin, cout)


def _torch_conv(x, w):
    """torch conv3d (cross-correlation, padding 1) on NDHWC data, weight
    [27, Cin, Cout] with tap t = 9 dz + 3 dy + dx."""
    xt = torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 0)))[None]
    wt = torch.from_numpy(np.ascontiguousarray(
        w.reshape(3, 3, 3, w.shape[1], w.shape[2]).transpose(4, 3, 0, 1, 2)))
    y = torch.nn.functional.conv3d(xt, wt, padding=1)[0]
    return np.moveaxis(y.numpy(), 0, -1)


@pytest.mark.parametrize("cin,cout", [(2, 16), (16, 16), (16, 1), (3, 5)])
def test_conv_matches_torch(orc, cin, cout):
    x = synthetic.uniform(1, 5 * 6 * 7 * cin).reshape(5, 6, 7, cin)
    w = _w(2, cin, cout)
    assert np.max(np.abs(orc.conv3d_fwd(x, w) - _torch_conv(x, w))) < 1e-12


def test_conv_with_stencil_taps_is_stencil(orc):
    """A 1->1 convolution with centre tap 6 and the six face taps -1 is the
    seven-point operator with zero Dirichlet ghosts (exact on integers)."""
    shape = (6, 7, 8)
    w = np.zeros((27, 1, 1))
    w[13] = 6.0
    for t in (4, 10, 12, 14, 16, 22):
        w[t] = -1.0
    x = synthetic.integers(3, 336, -100, 100).astype(np.float64)
    y = orc.conv3d_fwd(x.reshape(*shape, 1), w).reshape(-1)
    assert np.array_equal(y, orc.stencil_loops(x, shape))


def test_identity_kernel(orc):
    w = np.zeros((27, 4, 4))
    w[13] = np.eye(4)
    x = synthetic.uniform(4, 3 * 4 * 5 * 4).reshape(3, 4, 5, 4)
    assert np.array_equal(orc.conv3d_fwd(x, w), x)


def test_conv_backward_matches_torch(orc):
    x = synthetic.uniform(5, 4 * 5 * 6 * 3).reshape(4, 5, 6, 3)
    w = _w(6, 3, 4)
    dy = synthetic.uniform(7, 4 * 5 * 6 * 4).reshape(4, 5, 6, 4)
    dx, dw = orc.conv3d_bwd(x, w, dy)
    xt = torch.from_numpy(x.copy()).requires_grad_(True)
    wt = torch.from_numpy(w.copy()).requires_grad_(True)
    xc = xt.permute(3, 0, 1, 2)[None]
    wc = wt.reshape(3, 3, 3, 3, 4).permute(4, 3, 0, 1, 2)
    y = torch.nn.functional.conv3d(xc, wc, padding=1)[0].permute(1, 2, 3, 0)
    y.backward(torch.from_numpy(dy))
    assert np.max(np.abs(dx - xt.grad.numpy())) < 1e-12
    assert np.max(np.abs(dw - wt.grad.numpy())) < 1e-11


def _net(seed=10):
    chans = [2, 16, 16, 16, 1]
    return [_w(seed + i, chans[i], chans[i + 1], scale=(2.0 / (27 * chans[i])) ** 0.5 * 1.7)
            for i in range(4)]


def test_network_gradient_finite_differences(orc):
    """Central differences (h = 1e-6) on the full 2->16->16->16->1 network at 8^3."""
    n = 8
    ws = _net()
    inp = synthetic.uniform(20, n ** 3 * 2).reshape(n, n, n, 2)
    target = synthetic.uniform(21, n ** 3).reshape(n, n, n, 1)

    def loss_of(wlist):
        out, _ = orc.cnn_forward(wlist, inp)
        l, _ = orc.rel_mse([out], [target])
        return l

    out, acts = orc.cnn_forward(ws, inp)
    _, g = orc.rel_mse([out], [target])
    grads = orc.cnn_backward(ws, acts, g[0])
    rng = np.random.default_rng(0)
    h = 1e-6
    for li in range(4):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in ws[li].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[li][idx] += h
            wm[li][idx] -= h
            fd = (loss_of(wp) - loss_of(wm)) / (2 * h)
            an = grads[li][idx]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.max(np.abs(grads[li]))), (li, idx)


def test_network_gradient_matches_autograd(orc):
    n = 6
    ws = _net(30)
    inp = synthetic.uniform(31, n ** 3 * 2).reshape(n, n, n, 2)
    target = synthetic.uniform(32, n ** 3).reshape(n, n, n, 1)
    out, acts = orc.cnn_forward(ws, inp)
    _, g = orc.rel_mse([out], [target])
    grads = orc.cnn_backward(ws, acts, g[0])
    wt = [torch.from_numpy(w.copy()).requires_grad_(True) for w in ws]
    h = torch.from_numpy(inp).permute(3, 0, 1, 2)[None]
    for li, w in enumerate(wt):
        cin, cout = w.shape[1], w.shape[2]
        h = torch.nn.functional.conv3d(h, w.reshape(3, 3, 3, cin, cout).permute(4, 3, 0, 1, 2), padding=1)
        if li < 3:
            h = torch.relu(h)
    t = torch.from_numpy(target).permute(3, 0, 1, 2)[None]
    loss = ((h - t) ** 2).sum() / (t ** 2).sum()
    loss.backward()
    for li in range(4):
        assert np.max(np.abs(grads[li] - wt[li].grad.numpy())) <= 1e-10 * max(1.0, np.max(np.abs(grads[li])))


def test_linear_without_relu(orc):
    ws = _net(40)
    a = synthetic.uniform(41, 5 ** 3 * 2).reshape(5, 5, 5, 2)
    b = synthetic.uniform(42, 5 ** 3 * 2).reshape(5, 5, 5, 2)
    fa, _ = orc.cnn_forward(ws, a, relu=False)
    fb, _ = orc.cnn_forward(ws, b, relu=False)
    fab, _ = orc.cnn_forward(ws, 2.0 * a - 3.0 * b, relu=False)
    assert np.max(np.abs(fab - (2.0 * fa - 3.0 * fb))) < 1e-11


def test_adam_matches_torch(orc):
    w0 = synthetic.uniform(50, 100)
    grads = [synthetic.uniform(51 + s, 100) for s in range(5)]
    wt = torch.from_numpy(w0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(100), np.zeros(100)
    for s, g in enumerate(grads, start=1):
        wt.grad = torch.from_numpy(g.copy())
        opt.step()
        w, m, v = orc.adam(w, g, m, v, s)
    assert np.max(np.abs(w - wt.detach().numpy())) <= 1e-6 * np.max(np.abs(w))


def test_cnn_apply_scale_equivariance(orc):
    """z = rms(r) N(r / rms(r), g) is positively homogeneous of degree one in r."""
    shape = (5, 5, 5)
    ws = _net(60)
    r = synthetic.uniform(61, 125)
    g = synthetic.uniform(62, 125)
    z1 = orc.cnn_apply(ws, r, g, shape)
    z2 = orc.cnn_apply(ws, 4.0 * r, g, shape)
    assert np.max(np.abs(z2 - 4.0 * z1)) < 1e-12 * max(1.0, np.max(np.abs(z2)))


def test_anorm_loss_zero_at_optimum(orc):
    """The A-norm loss of z = D^-1 rh + pred vanishes at pred = eh - D^-1 rh."""
    shape = (5, 6, 7)
    n = 210
    k = synthetic.coefficient_field(7)[:n].astype(np.float64)  # any positive field
    rh, eh = synthetic.uniform(11, n), synthetic.uniform(12, n)
    dinv = 1.0 / orc.vdiag(k, shape)
    loss, grads = orc.anorm_loss([eh - dinv * rh], [rh], [eh], shape, kcell=k)
    assert abs(loss) < 1e-24 and np.max(np.abs(grads[0])) < 1e-12
    loss, _ = orc.anorm_loss([np.zeros(n)], [rh], [eh], shape, kcell=k)
    assert loss > 0.0


@pytest.mark.parametrize("mode", [(1, 1, 1), (2, 3, 1), (4, 5, 6)])
def test_anorm_loss_eigenvector_closed_form(orc, mode):
    """Constant coefficients, rh = lambda v and eh = v for a sine eigenvector v
    of A, pred = 0: u = (lambda/6 - 1) v, so L = (lambda - 6)^2 / (6 lambda)."""
    nz, ny, nx = 6, 7, 8
    a, b, c = mode
    v = synthetic.sine_mode(nx, ny, nz, a, b, c)
    lam = 6.0 - 2 * np.cos(a * np.pi / (nx + 1)) - 2 * np.cos(b * np.pi / (ny + 1)) - 2 * np.cos(c * np.pi / (nz + 1))
    loss, _ = orc.anorm_loss([np.zeros(v.size)], [lam * v], [v], (nz, ny, nx))
    assert abs(loss - (lam - 6.0) ** 2 / (6.0 * lam)) <= 1e-12 * max(1.0, loss)


@pytest.mark.parametrize("mode", [(1, 1, 1), (2, 3, 1), (4, 5, 6)])
def test_anorm_loss_energy_eigenvector_closed_form(orc, mode):
    """The energy normaliser on the same eigenvector pair: den = rh.eh =
    lambda |v|^2 and u.Au = (lambda/6 - 1)^2 lambda |v|^2, so L = (1 - lambda/6)^2;
    it also equals the relative A-norm error u.Au / eh.A eh."""
    nz, ny, nx = 6, 7, 8
    a, b, c = mode
    v = synthetic.sine_mode(nx, ny, nz, a, b, c)
    lam = 6.0 - 2 * np.cos(a * np.pi / (nx + 1)) - 2 * np.cos(b * np.pi / (ny + 1)) - 2 * np.cos(c * np.pi / (nz + 1))
    loss, _ = orc.anorm_loss([np.zeros(v.size)], [lam * v], [v], (nz, ny, nx), energy=True)
    assert abs(loss - (1.0 - lam / 6.0) ** 2) <= 1e-12 * max(1.0, loss)
    u = v / 6.0 * lam - v
    ref = float(np.dot(u, orc.stencil(u, (nz, ny, nx)))) / float(np.dot(v, orc.stencil(v, (nz, ny, nx))))
    assert abs(loss - ref) <= 1e-12 * max(1.0, loss)


@pytest.mark.parametrize("energy", [False, True])
def test_anorm_loss_gradient_finite_differences(orc, energy):
    shape = (3, 4, 5)
    n = 60
    k = np.exp(synthetic.uniform(21, n))
    rh, eh, p = synthetic.uniform(22, n), synthetic.uniform(23, n), synthetic.uniform(24, n)
    if energy:
        eh = np.abs(eh) * np.sign(rh)  # rh.eh > 0
    _, g = orc.anorm_loss([p], [rh], [eh], shape, kcell=k, energy=energy)
    h = 1e-6
    for j in (0, 7, 31, 59):
        dp = np.zeros(n)
        dp[j] = h
        lp, _ = orc.anorm_loss([p + dp], [rh], [eh], shape, kcell=k, energy=energy)
        lm, _ = orc.anorm_loss([p - dp], [rh], [eh], shape, kcell=k, energy=energy)
        assert abs((lp - lm) / (2 * h) - g[0][j]) <= 1e-6 * max(1.0, abs(g[0][j]))
