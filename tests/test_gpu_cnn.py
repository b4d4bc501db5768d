"""GPU parity of the learned preconditioner's network (MFMA implicit-GEMM
3x3x3 convolutions) and its training step against the FP64 oracle.

The GPU computes with BF16 weights and activations and FP32 accumulation.
The reference below composes the oracle's FP64 convolution with the same
BF16 roundings (weights, layer inputs, hidden outputs, back-propagated
gradients), so the remaining difference is FP32 accumulation order. Bars:
forward normwise relative error <= 1e-3; weight gradients <= 1e-2 per layer
(a gradient entry sums ~1e4 products and a few hidden values round to the
other BF16 neighbour); Adam <= 1e-6; the stencil-tap network is exact.
"""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

CHANS = [2, 16, 16, 16, 1]
OFF = [0, 864, 7776, 14688, 15120]


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _init_weights(seed):
    ws = []
    for i in range(4):
        cin, cout = CHANS[i], CHANS[i + 1]
        std = (2.0 / (27 * cin)) ** 0.5
        w = np.random.default_rng(seed + i).standard_normal((27, cin, cout)) * std
        ws.append(w.astype(np.float32).astype(np.float64))
    return ws


def _flat(ws):
    return np.concatenate([w.reshape(-1) for w in ws]).astype(np.float32)


def _fwd_emulated(orc, ws, inp, relu=True):
    """Oracle forward with the GPU's BF16 roundings; returns (out, acts)."""
    rb = orc.round_bf16
    wb = [rb(w) for w in ws]
    h = rb(inp)
    acts = [h]
    for li, w in enumerate(wb):
        h = orc.conv3d_fwd(h, w)
        if li < 3:
            h = rb(np.maximum(h, 0.0) if relu else h)
            acts.append(h)
    return h, acts, wb


def _bwd_emulated(orc, wb, acts, dout):
    """Oracle back-propagation with the GPU's BF16 roundings of the
    propagated gradients (the last layer's gradient enters both its weight
    gradient and the input-gradient convolution as BF16)."""
    rb = orc.round_bf16
    grads = [None] * 4
    g = dout
    for li in range(3, -1, -1):
        _, dw = orc.conv3d_bwd(acts[li], wb[li], rb(g) if li == 3 else g)
        grads[li] = dw
        if li > 0:
            gin = rb(g) if li == 3 else g
            dx, _ = orc.conv3d_bwd(acts[li], wb[li], gin)
            g = rb(dx * (acts[li] > 0.0))
    return grads


def _inputs(shape, seed):
    n = int(np.prod(shape))
    r = synthetic.uniform_f32(seed, n)
    g = synthetic.uniform_f32(seed + 1, n)
    return r, g


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 13, 20), (16, 16, 16), (5, 7, 3)])
def test_forward_raw(P, orc, shape):
    nz, ny, nx = shape
    ws = _init_weights(3)
    r, g = _inputs(shape, 10)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    z = torch.empty(r.size, dtype=torch.float32, device="cuda")
    P.cnn_forward(net, shape, torch.from_numpy(r).cuda(), torch.from_numpy(g).cuda(), z)
    inp = np.stack([r.reshape(shape), g.reshape(shape)], axis=-1).astype(np.float64)
    ref, _, _ = _fwd_emulated(orc, ws, inp)
    got = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref.reshape(-1)) / np.linalg.norm(ref)
    print(shape, "forward rel err", rel, flush=True)
    assert rel <= 1e-3


def test_forward_scaled(P, orc):
    """z = rms(r) N(r / rms(r), g) with ||r||^2 taken from a device scalar."""
    shape = (12, 12, 12)
    ws = _init_weights(5)
    r, g = _inputs(shape, 20)
    r = (r * 37.0).astype(np.float32)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    z = torch.empty(r.size, dtype=torch.float32, device="cuda")
    rr = torch.tensor([float(np.dot(r.astype(np.float64), r))], dtype=torch.float64, device="cuda")
    P.cnn_forward(net, shape, torch.from_numpy(r).cuda(), torch.from_numpy(g).cuda(), z, rr=rr)
    rho = np.sqrt(rr.item() / r.size)
    inp = np.stack([(r / np.float32(rho)).reshape(shape), g.reshape(shape)], axis=-1).astype(np.float64)
    ref, _, _ = _fwd_emulated(orc, ws, inp)
    got = z.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - rho * ref.reshape(-1)) <= 1e-3 * np.linalg.norm(rho * ref)


@pytest.mark.parametrize("scaled", [False, True])
def test_forward_input_dtypes(P, scaled):
    """The first layer forms its input from r itself: r given as FP64 or BF16
    holding the same values as an FP32 r (BF16-representable values) gives
    bit-identical outputs, with and without the rms scaling."""
    shape = (9, 13, 20)
    n = int(np.prod(shape))
    ws = _init_weights(7)
    r, g = _inputs(shape, 30)
    bits = synthetic.f32_to_bf16_bits(r * 5.0)
    r32 = (bits.astype(np.uint32) << 16).view(np.float32)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    gd = torch.from_numpy(g).cuda()
    rr = torch.tensor([float(np.dot(r32.astype(np.float64), r32))], dtype=torch.float64, device="cuda") if scaled else None
    outs = []
    for rt in (torch.from_numpy(r32).cuda(), torch.from_numpy(r32.astype(np.float64)).cuda(),
               torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)):
        z = torch.empty(n, dtype=torch.float32, device="cuda")
        P.cnn_forward(net, shape, rt, gd, z, rr=rr)
        outs.append(z.cpu().numpy())
    assert np.abs(outs[0]).max() > 0
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    assert np.array_equal(outs[0].view(np.uint32), outs[2].view(np.uint32))


def test_forward_unaligned_output(P):
    """The last layer stores four voxels per lane with one 16-byte store when
    the output row allows it; an output pointer off 16-byte alignment takes
    the element-wise path and must give the same bits."""
    shape = (12, 16, 32)
    n = int(np.prod(shape))
    ws = _init_weights(11)
    r, g = _inputs(shape, 40)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    rd, gd = torch.from_numpy(r).cuda(), torch.from_numpy(g).cuda()
    za = torch.empty(n, dtype=torch.float32, device="cuda")
    P.cnn_forward(net, shape, rd, gd, za)
    zfull = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    zu = zfull[1:]
    assert zu.data_ptr() % 16 != 0
    P.cnn_forward(net, shape, rd, gd, zu)
    assert float(zfull[0]) == 0.0
    assert np.array_equal(za.cpu().numpy().view(np.uint32), zu.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("n", [64, 128])
def test_forward_full_size_sampled(P, orc, n):
    """The scaled forward at the learned-preconditioner workload's grid sizes
    (g the standardised Gaussian random field), checked at sampled voxels:
    the output at p depends only on inputs within 4 voxels of p (four 3x3x3
    layers), so the oracle runs on that window clipped to the grid, whose
    cut faces lie outside every intermediate value the output needs."""
    shape = (n, n, n)
    N = n ** 3
    ws = _init_weights(11)
    r = synthetic.uniform_f32(30, N)
    g = synthetic.gaussian_random_field(n).astype(np.float32)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    z = torch.empty(N, dtype=torch.float32, device="cuda")
    rr = torch.tensor([float(np.dot(r.astype(np.float64), r))], dtype=torch.float64, device="cuda")
    P.cnn_forward(net, shape, torch.from_numpy(r).cuda(), torch.from_numpy(g).cuda(), z, rr=rr)
    got_all = z.cpu().numpy().astype(np.float64).reshape(shape)
    rho = np.sqrt(rr.item() / N)
    r3 = (r / np.float32(rho)).reshape(shape)
    g3 = g.reshape(shape)
    rng = np.random.default_rng(31)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5), (n // 2, 0, n - 1), (3, 7, 15), (4, 8, 16)]
    pts += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(18)]
    got, ref = [], []
    for p in pts:
        lo = [max(0, c - 4) for c in p]
        hi = [min(n, c + 5) for c in p]
        win = tuple(slice(a, b) for a, b in zip(lo, hi))
        inp = np.stack([r3[win], g3[win]], axis=-1).astype(np.float64)
        out, _, _ = _fwd_emulated(orc, ws, inp)
        ref.append(rho * out[tuple(c - a for c, a in zip(p, lo))][0])
        got.append(got_all[p])
    got, ref = np.array(got), np.array(ref)
    err = np.abs(got - ref)
    print(n, "sampled forward max abs err", err.max(), "rms ref", np.sqrt(np.mean(ref ** 2)), flush=True)
    assert np.linalg.norm(err) <= 1e-3 * np.linalg.norm(ref)
    assert err.max() <= 5e-3 * np.abs(ref).max()
    assert np.isfinite(got_all).all()


def test_stencil_network_exact(P, orc):
    """A network that carries r through ReLU as (relu(r), relu(-r)) and applies
    the seven-point taps in its last layer computes A r exactly on integers
    (|r| <= 16 is exact in BF16 and every partial sum is an integer)."""
    shape = (10, 11, 12)
    ws = [np.zeros((27, CHANS[i], CHANS[i + 1])) for i in range(4)]
    ws[0][13, 0, 0], ws[0][13, 0, 1] = 1.0, -1.0
    for li in (1, 2):
        ws[li][13, 0, 0] = ws[li][13, 1, 1] = 1.0
    for t, v in ((13, 6.0), (4, -1.0), (10, -1.0), (12, -1.0), (14, -1.0), (16, -1.0), (22, -1.0)):
        ws[3][t, 0, 0], ws[3][t, 1, 0] = v, -v
    n = int(np.prod(shape))
    r = synthetic.integers(7, n, -16, 16)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    P.cnn_forward(net, shape, torch.from_numpy(r).cuda(), torch.zeros(n, device="cuda"), z)
    assert np.array_equal(z.cpu().numpy().astype(np.float64), orc.stencil(r.astype(np.float64), shape))


@pytest.mark.parametrize("shape,batch", [((8, 8, 8), 1), ((10, 9, 12), 2)])
def test_loss_and_gradients(P, orc, shape, batch):
    n = int(np.prod(shape))
    ws = _init_weights(11)
    g = synthetic.uniform_f32(40, n)
    pairs = []
    for b in range(batch):
        rh = synthetic.f32_to_bf16_bits(synthetic.uniform_f32(50 + b, n))
        eh = synthetic.f32_to_bf16_bits(synthetic.uniform_f32(60 + b, n))
        pairs += [rh, eh]
    pairs_np = np.concatenate(pairs)
    from gpu_helpers import bf16_tensor

    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    grad = torch.zeros(P.cnn_num_weights(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.cnn_loss_grad(net, shape, bf16_tensor(pairs_np).cuda(), torch.from_numpy(g).cuda(), batch, grad=grad, loss=loss)
    # oracle: mean over the batch of the relative MSE and its gradient
    ref_loss, ref_grads = 0.0, [np.zeros((27, CHANS[i], CHANS[i + 1])) for i in range(4)]
    for b in range(batch):
        rh = synthetic.bf16_bits_to_f32(pairs[2 * b]).astype(np.float64)
        eh = synthetic.bf16_bits_to_f32(pairs[2 * b + 1]).astype(np.float64)
        inp = np.stack([rh.reshape(shape), g.astype(np.float64).reshape(shape)], axis=-1)
        out, acts, wb = _fwd_emulated(orc, ws, inp)
        l, dl = orc.rel_mse([out], [eh.reshape(*shape, 1)])
        ref_loss += l / batch
        gr = _bwd_emulated(orc, wb, acts, dl[0])
        for i in range(4):
            ref_grads[i] += gr[i] / batch
    assert abs(loss.item() - ref_loss) <= 1e-3 * ref_loss
    gg = grad.cpu().numpy().astype(np.float64)
    for i in range(4):
        got = gg[OFF[i]:OFF[i + 1]].reshape(ref_grads[i].shape)
        rel = np.linalg.norm(got - ref_grads[i]) / np.linalg.norm(ref_grads[i])
        print(shape, "layer", i + 1, "grad rel err", rel, flush=True)
        assert rel <= 1e-2


@pytest.mark.parametrize("var,energy", [(False, False), (True, False), (True, True)])
def test_anorm_loss_and_gradients(P, orc, var, energy):
    """A-norm loss of the Jacobi-plus-correction preconditioner (operator from
    an F32 context) against the oracle's anorm_loss with the GPU's BF16
    roundings emulated, with either normaliser; same bars as the
    relative-MSE test."""
    shape = (10, 9, 12)
    nz, ny, nx = shape
    n = int(np.prod(shape))
    batch = 2
    ws = _init_weights(13)
    g = synthetic.uniform_f32(41, n)
    k32 = synthetic.coefficient_field(12)[:n].copy() if var else None
    pairs = []
    for b in range(batch):
        rr = synthetic.uniform_f32(52 + b, n)
        ee = synthetic.uniform_f32(62 + b, n)
        if energy:
            ee = (np.abs(ee) * np.sign(rr)).astype(np.float32)  # rh.eh > 0
        pairs += [synthetic.f32_to_bf16_bits(rr), synthetic.f32_to_bf16_bits(ee)]
    from gpu_helpers import bf16_tensor

    ctx = P.pcg_create(nx, ny, nz, torch.float32)
    if var:
        P.pcg_set_coefficients(ctx, torch.from_numpy(k32).cuda())
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    P.cnn_set_operator(net, ctx)
    P.cnn_set_loss_norm(net, 1 if energy else 0)
    grad = torch.zeros(P.cnn_num_weights(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.cnn_loss_grad(net, shape, bf16_tensor(np.concatenate(pairs)).cuda(), torch.from_numpy(g).cuda(), batch,
                    grad=grad, loss=loss)
    k64 = None if k32 is None else k32.astype(np.float64)
    ref_loss, ref_grads = 0.0, [np.zeros((27, CHANS[i], CHANS[i + 1])) for i in range(4)]
    for b in range(batch):
        rh = synthetic.bf16_bits_to_f32(pairs[2 * b]).astype(np.float64)
        eh = synthetic.bf16_bits_to_f32(pairs[2 * b + 1]).astype(np.float64)
        inp = np.stack([rh.reshape(shape), g.astype(np.float64).reshape(shape)], axis=-1)
        out, acts, wb = _fwd_emulated(orc, ws, inp)
        l, dl = orc.anorm_loss([out.reshape(-1)], [rh], [eh], shape, kcell=k64, energy=energy)
        ref_loss += l / batch
        gr = _bwd_emulated(orc, wb, acts, dl[0].reshape(*shape, 1))
        for i in range(4):
            ref_grads[i] += gr[i] / batch
    print("anorm loss", loss.item(), ref_loss, flush=True)
    assert abs(loss.item() - ref_loss) <= 1e-3 * ref_loss
    gg = grad.cpu().numpy().astype(np.float64)
    for i in range(4):
        got = gg[OFF[i]:OFF[i + 1]].reshape(ref_grads[i].shape)
        rel = np.linalg.norm(got - ref_grads[i]) / np.linalg.norm(ref_grads[i])
        print("anorm layer", i + 1, "grad rel err", rel, flush=True)
        assert rel <= 1e-2
    # the operator can be unset again (relative MSE)
    P.cnn_set_operator(net, None)


def test_adam_step(P, orc):
    ws = _init_weights(21)
    w0 = _flat(ws)
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(w0).cuda())
    w, m, v = w0.astype(np.float64), np.zeros(w0.size), np.zeros(w0.size)
    for step in range(1, 4):
        gr = synthetic.uniform_f32(70 + step, w0.size) * 1e-2
        P.cnn_adam_step(net, torch.from_numpy(gr).cuda(), lr=1e-3)
        w, m, v = orc.adam(w, gr.astype(np.float64), m, v, step)
    got = P.cnn_get_weights(net).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - w)) <= 1e-6 * np.max(np.abs(w))


def test_training_reduces_loss(P):
    """A few Adam steps on a fixed batch reduce the loss."""
    shape = (16, 16, 16)
    n = int(np.prod(shape))
    ws = _init_weights(31)
    g = synthetic.uniform_f32(80, n)
    r = synthetic.uniform_f32(81, n)
    from gpu_helpers import bf16_tensor

    # target: a smooth function of r (its 6-neighbour average), learnable by the network
    rr = r.reshape(shape).astype(np.float64)
    e = (np.roll(rr, 1, 0) + np.roll(rr, -1, 0) + np.roll(rr, 1, 1) + np.roll(rr, -1, 1) + np.roll(rr, 1, 2)
         + np.roll(rr, -1, 2)) / 6.0
    pairs = np.concatenate([synthetic.f32_to_bf16_bits(r), synthetic.f32_to_bf16_bits(e.reshape(-1).astype(np.float32))])
    pt = bf16_tensor(pairs).cuda()
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(ws)).cuda())
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    for _ in range(30):
        P.cnn_train_step(net, shape, pt, torch.from_numpy(g).cuda(), 1, lr=3e-3, loss=loss)
        losses.append(loss.item())
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_adam_checkpoint_resume(P, tmp_path):
    """Weights plus Adam's moments and step count restore training exactly:
    resuming from a checkpoint (in memory, or through a checkpoint file)
    reproduces the uninterrupted run bit for bit (the training kernels reduce
    in a fixed order, with no atomics)."""
    shape = (16, 16, 16)
    n = int(np.prod(shape))
    from gpu_helpers import bf16_tensor

    g = torch.from_numpy(synthetic.uniform_f32(90, n)).cuda()
    pairs = np.concatenate([synthetic.f32_to_bf16_bits(synthetic.uniform_f32(91, n)),
                            synthetic.f32_to_bf16_bits(synthetic.uniform_f32(92, n))])
    pt = bf16_tensor(pairs).cuda()
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(_flat(_init_weights(41))).cuda())
    for _ in range(2):
        P.cnn_train_step(net, shape, pt, g, 1, lr=3e-3)
    w_ck = P.cnn_get_weights(net).clone()
    m_ck, v_ck, step_ck = P.cnn_get_adam(net)
    from paper_2603_23343_amd import checkpoint

    ck_path = str(tmp_path / "net.ckpt")
    checkpoint.save(net, ck_path, meta={"steps": 2})
    assert step_ck == 2
    assert torch.count_nonzero(v_ck) > 0
    for _ in range(2):
        P.cnn_train_step(net, shape, pt, g, 1, lr=3e-3)
    w_ref = P.cnn_get_weights(net).cpu()

    # a second network resumes from the checkpoint
    net2 = P.cnn_create()
    P.cnn_set_weights(net2, w_ck)
    P.cnn_set_adam(net2, m_ck, v_ck, step_ck)
    for _ in range(2):
        P.cnn_train_step(net2, shape, pt, g, 1, lr=3e-3)
    assert torch.equal(P.cnn_get_weights(net2).cpu(), w_ref)
    assert P.cnn_get_adam(net2)[2] == 4

    # the same through the checkpoint file
    net4 = P.cnn_create()
    assert checkpoint.load(net4, ck_path) == {"steps": 2}
    for _ in range(2):
        P.cnn_train_step(net4, shape, pt, g, 1, lr=3e-3)
    assert torch.equal(P.cnn_get_weights(net4).cpu(), w_ref)

    # without the moments (set_weights resets them) the run differs
    net3 = P.cnn_create()
    P.cnn_set_weights(net3, w_ck)
    for _ in range(2):
        P.cnn_train_step(net3, shape, pt, g, 1, lr=3e-3)
    assert not torch.equal(P.cnn_get_weights(net3).cpu(), w_ref)
    with pytest.raises(RuntimeError):
        P.cnn_set_adam(net3, m_ck, v_ck, -1)
