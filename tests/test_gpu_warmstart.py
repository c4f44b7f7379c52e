"""GPU checks of the learned warm start: BF16-MFMA kernels against the FP64
reference network, training progress, and the solver's fallback start."""

import ctypes as C
import os

import numpy as np
import pytest
import torch

from gpu_common import make_pair, rel, say, to_dev, to_np
from oracle import cisor as ocisor
from oracle import net as onet
from synth import complex_normal, disks_2d, mixed_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# tile: 0 automatic (the last two shapes take the two-tiles-per-block launch), 1..6 = 256x128, 128x128, 256x64, 128x64, 256x32, 128x32 (pixels x channels)
@pytest.mark.parametrize("B,H,W,Ci,Co,tile", [(2, 16, 16, 32, 32, 0), (1, 32, 24, 64, 96, 0), (4, 8, 8, 96, 32, 0),
                                              (2, 16, 16, 64, 128, 1), (1, 16, 16, 32, 128, 2),
                                              (2, 16, 16, 128, 64, 3), (1, 16, 8, 96, 64, 4),
                                              (1, 16, 16, 64, 96, 5), (4, 16, 8, 32, 256, 1),
                                              (16, 128, 128, 32, 32, 0), (16, 128, 128, 32, 64, 0)])
def test_conv3x3_forward_matches_fp64(B, H, W, Ci, Co, tile):
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    say(f"conv fwd {B}x{H}x{W} {Ci}->{Co} tile {tile}")
    g = torch.Generator().manual_seed(B * H + Ci)
    x = torch.randn(B, H, W, Ci, generator=g).to(torch.bfloat16)
    w = (torch.randn(9, Co, Ci, generator=g) / (3 * Ci ** 0.5)).to(torch.bfloat16)
    b = torch.randn(Co, generator=g).float()
    ref = onet.conv3x3(x.double().permute(0, 3, 1, 2), w.double().reshape(3, 3, Co, Ci).permute(2, 3, 0, 1),
                       b.double()).permute(0, 2, 3, 1)
    xd, wd, bd = x.cuda(), w.cuda(), b.cuda()
    y32 = torch.empty(B, H, W, Co, dtype=torch.float32, device="cuda")
    assert lib.cisor_nn_conv3x3(_ptr(xd), _ptr(wd), _ptr(bd), _ptr(y32), B, H, W, Ci, Co, 0, 1, tile, _stream()) == 0
    yb = torch.empty(B, H, W, Co, dtype=torch.bfloat16, device="cuda")
    assert lib.cisor_nn_conv3x3(_ptr(xd), _ptr(wd), _ptr(bd), _ptr(yb), B, H, W, Ci, Co, 1, 0, tile, _stream()) == 0
    torch.cuda.synchronize()
    assert rel(y32.cpu().double().numpy(), ref.numpy()) < 1e-5          # FP32 accumulation of exact products
    assert rel(yb.cpu().double().numpy(), torch.relu(ref).numpy()) < 8e-3   # BF16 output rounding


@pytest.mark.parametrize("B,H,W,Ci,Co", [(2, 16, 16, 32, 32), (1, 32, 32, 64, 32)])
def test_conv3x3_weight_gradient_matches_fp64(B, H, W, Ci, Co):
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    g = torch.Generator().manual_seed(7 + Ci)
    x = torch.randn(B, H, W, Ci, generator=g).to(torch.bfloat16)
    dy = torch.randn(B, H, W, Co, generator=g).to(torch.bfloat16)
    ref = torch.nn.grad.conv2d_weight(x.double().permute(0, 3, 1, 2), (Co, Ci, 3, 3),
                                      dy.double().permute(0, 3, 1, 2), padding=1)   # [Co, Ci, 3, 3]
    ref = ref.permute(2, 3, 0, 1).reshape(9, Co, Ci)
    dw = torch.empty(9, Co, Ci, dtype=torch.float32, device="cuda")
    scratch = torch.empty(8 * 9 * Co * Ci, dtype=torch.float32, device="cuda")
    assert lib.cisor_nn_conv3x3_wgrad(_ptr(x.cuda()), _ptr(dy.cuda()), _ptr(dw), _ptr(scratch), B, H, W, Ci, Co, 8,
                                      _stream()) == 0
    torch.cuda.synchronize()
    assert rel(dw.cpu().double().numpy(), ref.numpy()) < 1e-5


@pytest.mark.parametrize("B,H,W,C1,C2,Co,tile", [(2, 16, 16, 32, 64, 32, 0), (1, 32, 16, 64, 128, 64, 0),
                                                  (4, 8, 8, 128, 256, 128, 0), (2, 16, 16, 32, 32, 64, 3),
                                                  (1, 16, 16, 64, 32, 96, 5)])
def test_conv3x3_on_concatenation_in_place_is_bit_identical(B, H, W, C1, C2, Co, tile):
    """The decoder convolution that reads [x | up2(x2)] in place gives the same
    bits as the plain convolution on the formed concatenation."""
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    say(f"conv cat {B}x{H}x{W} {C1}+{C2}->{Co} tile {tile}")
    g = torch.Generator().manual_seed(B * H + C1 + C2)
    x = torch.randn(B, H, W, C1, generator=g).to(torch.bfloat16)
    x2 = torch.randn(B, H // 2, W // 2, C2, generator=g).to(torch.bfloat16)
    Ci = C1 + C2
    w = (torch.randn(9, Co, Ci, generator=g) / (3 * Ci ** 0.5)).to(torch.bfloat16)
    b = torch.randn(Co, generator=g).float()
    cat = torch.cat([x, x2.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)], dim=3).contiguous()
    xd, x2d, catd, wd, bd = x.cuda(), x2.cuda(), cat.cuda(), w.cuda(), b.cuda()
    for relu, out_f32, dt in ((0, 1, torch.float32), (1, 0, torch.bfloat16)):
        ya = torch.empty(B, H, W, Co, dtype=dt, device="cuda")
        yb = torch.empty(B, H, W, Co, dtype=dt, device="cuda")
        assert lib.cisor_nn_conv3x3(_ptr(catd), _ptr(wd), _ptr(bd), _ptr(ya), B, H, W, Ci, Co, relu, out_f32, tile,
                                    _stream()) == 0
        assert lib.cisor_nn_conv3x3_ex(_ptr(xd), _ptr(x2d), C1, _ptr(wd), _ptr(bd), _ptr(yb), B, H, W, Ci, Co, relu,
                                       out_f32, tile, 1, None, 0, _stream()) == 0
        torch.cuda.synchronize()
        assert torch.equal(ya, yb)
    y = torch.empty(B, H, W, Co, dtype=torch.float32, device="cuda")
    bad = [(C1 + 8, H, W), (Ci, H, W), (C1, H + 1, W)]      # C1 not a slice multiple, no second part, odd height
    for c1, h, ww in bad:
        assert lib.cisor_nn_conv3x3_ex(_ptr(xd), _ptr(x2d), c1, _ptr(wd), _ptr(bd), _ptr(y), B, h, ww, Ci, Co, 0, 1,
                                       tile, 1, None, 0, _stream()) == _lib.E_ARG


@pytest.mark.parametrize("B,H,W,Ci,Co,splits,cat", [(2, 8, 8, 256, 256, 8, False), (1, 16, 16, 128, 128, 4, False),
                                                    (4, 8, 8, 384, 128, 3, True), (2, 16, 16, 96, 32, 2, True),
                                                    (1, 8, 16, 32, 64, 9, False)])
def test_conv3x3_split_k_matches_fp64_and_the_unsplit_launch(B, H, W, Ci, Co, splits, cat):
    """Split K: the FP32 partials of `splits` blocks summed in split order
    equal the FP64 convolution and the unsplit launch to FP32 rounding."""
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    say(f"conv split-K {B}x{H}x{W} {Ci}->{Co} splits {splits} cat {cat}")
    g = torch.Generator().manual_seed(B + H + Ci + splits)
    C1 = Ci // 3 // 32 * 32 if cat else 0
    x = torch.randn(B, H, W, Ci, generator=g).to(torch.bfloat16)
    if cat:   # the same input given as [skip | up2(low)]
        low = torch.randn(B, H // 2, W // 2, Ci - C1, generator=g).to(torch.bfloat16)
        x = torch.cat([x[..., :C1], low.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)], dim=3).contiguous()
    w = (torch.randn(9, Co, Ci, generator=g) / (3 * Ci ** 0.5)).to(torch.bfloat16)
    b = torch.randn(Co, generator=g).float()
    ref = onet.conv3x3(x.double().permute(0, 3, 1, 2), w.double().reshape(3, 3, Co, Ci).permute(2, 3, 0, 1),
                       b.double()).permute(0, 2, 3, 1)
    xd = (x[..., :C1].contiguous() if cat else x).cuda()
    x2d = low.cuda() if cat else None
    wd, bd = w.cuda(), b.cuda()
    ws = torch.empty(splits * B * H * W * Co, dtype=torch.float32, device="cuda")
    y1 = torch.empty(B, H, W, Co, dtype=torch.float32, device="cuda")
    ys = torch.empty_like(y1)
    args = (_ptr(xd), _ptr(x2d), C1, _ptr(wd), _ptr(bd))
    assert lib.cisor_nn_conv3x3_ex(*args, _ptr(y1), B, H, W, Ci, Co, 0, 1, 0, 1, None, 0, _stream()) == 0
    assert lib.cisor_nn_conv3x3_ex(*args, _ptr(ys), B, H, W, Ci, Co, 0, 1, 0, splits, _ptr(ws), ws.numel(),
                                   _stream()) == 0
    yb = torch.empty(B, H, W, Co, dtype=torch.bfloat16, device="cuda")
    assert lib.cisor_nn_conv3x3_ex(*args, _ptr(yb), B, H, W, Ci, Co, 1, 0, 0, splits, _ptr(ws), ws.numel(),
                                   _stream()) == 0
    torch.cuda.synchronize()
    assert rel(ys.cpu().double().numpy(), ref.numpy()) < 1e-5
    assert rel(ys.cpu().double().numpy(), y1.cpu().double().numpy()) < 1e-6
    assert rel(yb.cpu().double().numpy(), torch.relu(ref).numpy()) < 8e-3
    # a split needs a workspace of splits x B H W x Co floats
    assert lib.cisor_nn_conv3x3_ex(*args, _ptr(ys), B, H, W, Ci, Co, 0, 1, 0, 2, None, 0, _stream()) == _lib.E_ARG
    assert lib.cisor_nn_conv3x3_ex(*args, _ptr(ys), B, H, W, Ci, Co, 0, 1, 0, 2, _ptr(ws), B * H * W * Co,
                                   _stream()) == _lib.E_ARG


def _net_inputs(n=64, B=8, seed=0):
    rng = np.random.default_rng(seed)
    f = np.stack([mixed_2d(n, seed + i).ravel() for i in range(B)])
    th = 2 * np.pi * rng.uniform(size=B)
    xs = (np.arange(n) - (n - 1) / 2) * 0.1
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    uin = np.stack([np.exp(2j * np.pi * (np.cos(t) * X + np.sin(t) * Y)).ravel() for t in th])
    u = uin * (1 + 0.3 * f) + 0.2j * f
    return f, uin, u


def test_network_forward_and_gradient_match_fp64_reference():
    """Whole network: prediction and parameter gradient of the relative-L2 loss
    against the FP64 autograd reference with the same parameters (BF16 bar)."""
    from paper_1708_01663_amd.warmstart import WarmStartNet
    say("net vs fp64")
    n, B = 64, 8
    net = WarmStartNet(n, n, 32, max_batch=B, seed=3)
    p = net.params().cpu().numpy()
    p[-32:] = np.random.default_rng(0).standard_normal(32) * 0.05    # non-zero head bias
    net.set_params(p)
    f, uin, u = _net_inputs(n, B)
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    ud = torch.tensor(uin, dtype=torch.complex64, device="cuda")
    tgt = torch.tensor(u, dtype=torch.complex64, device="cuda")
    ub = 0.3 * complex_normal(uin.shape, 9)          # stands in for the first-Born scattered field
    bd = torch.tensor(ub, dtype=torch.complex64, device="cuda")
    u0 = net.predict(fd, ud, bd).cpu().numpy()
    ref = onet.predict(p, f, uin, n, n, u_born=ub)
    assert rel(u0 - uin, ref - uin) < 3e-2
    assert rel(net.predict(fd, ud).cpu().numpy() - uin, onet.predict(p, f, uin, n, n) - uin) < 3e-2
    L, g = net.loss_grad(fd, ud, tgt, u_born=bd)
    Lr, gr = onet.loss_and_grad(p, f, uin, u, n, n, u_born=ub)
    assert abs(L - Lr) < 3e-2 * Lr
    assert rel(g.cpu().numpy(), gr) < 5e-2
    # per layer, the weight gradients agree in direction
    off = 0
    for ci, co, _ in onet.layer_specs(32):
        k = 9 * ci * co
        a, b = g.cpu().numpy()[off:off + k], gr[off:off + k]
        if np.linalg.norm(b) > 0:
            assert np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)) > 0.99
        off += k + co


@pytest.mark.parametrize("n,B", [(64, 8), (128, 16)])
def test_inference_forward_equals_the_training_forward(n, B):
    """cisor_net_forward (network input, pooling and output formed inside the
    convolutions, decoder inputs read in place) and the loss path (every
    intermediate materialised) compute the same network output: the relative-L2
    loss of the prediction equals the loss the training call reports.  At 64^2
    the bottleneck is too narrow for the tiled kernel and takes the unfused
    kernels; at 128^2 every fused form runs."""
    from paper_1708_01663_amd.warmstart import WarmStartNet
    say(f"inference vs training forward {n}^2 x {B}")
    net = WarmStartNet(n, n, 32, max_batch=B, seed=5)
    f, uin, u = _net_inputs(n, B, seed=2)
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    ud = torch.tensor(uin, dtype=torch.complex64, device="cuda")
    tgt = torch.tensor(u, dtype=torch.complex64, device="cuda")
    bd = torch.tensor(0.3 * complex_normal(uin.shape, 3), dtype=torch.complex64, device="cuda")
    out = (net.predict(fd, ud, bd) - ud).cpu().numpy().astype(np.complex128)
    t = (tgt - ud).cpu().numpy().astype(np.complex128)
    L_pred = np.mean(np.sum(np.abs(out - t) ** 2, axis=1) / np.sum(np.abs(t) ** 2, axis=1))
    L, _ = net.loss_grad(fd, ud, tgt, u_born=bd)
    assert abs(L - L_pred) <= 1e-5 * L


def test_fused_inference_at_the_workload_size_matches_fp64_reference():
    """The inference forward at 128^2 x 16 (every fused form and the
    two-tiles-per-block launch) against the FP64 reference network."""
    from paper_1708_01663_amd.warmstart import WarmStartNet
    say("fused inference vs fp64 at 128^2 x 16")
    n, B = 128, 16
    net = WarmStartNet(n, n, 32, max_batch=B, seed=7)
    p = net.params().cpu().numpy()
    p[-32:] = np.random.default_rng(1).standard_normal(32) * 0.05
    net.set_params(p)
    f, uin, _ = _net_inputs(n, B, seed=6)
    ub = 0.3 * complex_normal(uin.shape, 11)
    u0 = net.predict(torch.tensor(f, dtype=torch.float32, device="cuda"),
                     torch.tensor(uin, dtype=torch.complex64, device="cuda"),
                     torch.tensor(ub, dtype=torch.complex64, device="cuda")).cpu().numpy()
    ref = onet.predict(p, f, uin, n, n, u_born=ub)
    assert rel(u0 - uin, ref - uin) < 3e-2


def test_training_reduces_loss():
    from paper_1708_01663_amd.warmstart import WarmStartNet
    n, B = 64, 8
    net = WarmStartNet(n, n, 32, max_batch=B, seed=1)
    f, uin, u = _net_inputs(n, B, seed=4)
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    ud = torch.tensor(uin, dtype=torch.complex64, device="cuda")
    tgt = torch.tensor(u, dtype=torch.complex64, device="cuda")
    first = net.train_step(fd, ud, tgt, 1e-3)
    for _ in range(60):
        last = net.train_step(fd, ud, tgt, 1e-3)
    assert last < 0.5 * first


def test_fallback_start_keeps_the_better_guess():
    """start = 3: a guess worse than the first-Born field falls back to it; the
    converged solution as guess is kept and needs (almost) no iterations."""
    from paper_1708_01663_amd.cisor import SolveOpts
    n, h, T = 64, 1 / 10, 4
    prob, op = make_pair(n, h, T, 8)
    f = disks_2d(n, 2, count=3, radius_px=(5, 12), eps_range=(1.2, 1.6))
    fd = to_dev(f.ravel(), op, real=True)
    u, _, its_born, _ = op.forward(fd, SolveOpts(tol=1e-6, start=1), project=False)
    guess = u.clone()
    guess[1] = 10.0 * guess[1]          # a bad guess for transmitter 1
    u2, _, its, code = op.forward(fd, SolveOpts(tol=1e-6, start=3), u0=guess, project=False)
    assert code == 0
    choice = (C.c_int * T)()
    assert op.lib.cisor_get_start_choice(op.handle, choice) == 0
    assert list(choice) == [0, 1, 0, 0]
    assert its[1] == its_born[1]
    assert max(its[0], its[2], its[3]) <= 2
    u_ref, _ = ocisor.forward(prob, f, tol=1e-10)
    assert rel(to_np(u2).reshape(T, n, n), u_ref) < 1e-4


def test_zero_fallback_start_keeps_the_better_guess():
    """start = 5: a guess whose starting residual exceeds ||b|| (a scaled
    solution, or one with a non-finite entry) is replaced by the zero start
    (the same iterations as a zero-start solve); the converged solution as a
    guess is kept and needs (almost) no iterations; every field matches the
    oracle's solve."""
    from paper_1708_01663_amd.cisor import SolveOpts
    n, h, T = 64, 1 / 10, 4
    prob, op = make_pair(n, h, T, 8)
    f = disks_2d(n, 2, count=3, radius_px=(5, 12), eps_range=(1.2, 1.6))
    fd = to_dev(f.ravel(), op, real=True)
    u, _, its_zero, _ = op.forward(fd, SolveOpts(tol=1e-6, start=0), project=False)
    guess = u.clone()
    guess[1] = 10.0 * guess[1]          # starting residual 9 ||b||
    guess[2, 17] = float("nan")         # non-finite starting residual
    u2, _, its, code = op.forward(fd, SolveOpts(tol=1e-6, start=5), u0=guess, project=False)
    assert code == 0
    choice = (C.c_int * T)()
    assert op.lib.cisor_get_start_choice(op.handle, choice) == 0
    assert list(choice) == [0, 1, 1, 0]
    assert its[1] == its_zero[1] and its[2] == its_zero[2]
    assert max(its[0], its[3]) <= 2
    u_ref, _ = ocisor.forward(prob, f, tol=1e-10)
    assert rel(to_np(u2).reshape(T, n, n), u_ref) < 1e-4


def test_born_field_matches_oracle():
    """cisor_born_field: G diag(f) u_in,t = u_in,t - A u_in,t (eq. A_def) for
    every transmitter, against the oracle's operator."""
    from oracle import operators
    for n, prec, bar in ((48, "c64", 2e-6), (33, "c128", 1e-12)):
        prob, op = make_pair(n, 1 / 10, 3, 8, precision=prec)
        f = disks_2d(n, 5, count=3, radius_px=(4, 9), eps_range=(1.1, 1.9))
        ub = to_np(op.born_field(to_dev(f.ravel(), op, real=True))).reshape(3, n, n)
        ref = np.stack([prob.u_in[t] - operators.apply_A(prob.Ghat, f, prob.u_in[t]) for t in range(3)])
        assert rel(ub, ref) < bar, (n, prec)


def test_trained_network_starts_closer_than_zero_and_born():
    """The committed weights (trained on the GPU by the library's own kernels on
    solver-generated fields) on held-out phantoms: the network start needs fewer
    LS iterations to the same true residual than the zero and first-Born starts,
    its field error is well below that of the first-Born start (1.0 by
    definition), and the per-system fallback rarely triggers."""
    from paper_1708_01663_amd import warmstart
    if not os.path.exists(warmstart.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    say("trained warm start")
    op = warmstart.make_op()
    net = warmstart.WarmStartNet.load(warmstart.DEFAULT_WEIGHTS)
    res = warmstart.evaluate(op, net, range(300000, 300008))
    say(str(res))
    assert res["net"]["mean_iters"] < 0.97 * res["born"]["mean_iters"]
    assert res["net"]["mean_iters"] < res["zero"]["mean_iters"]
    assert res["net_rel_error_of_scattered_field"] < 0.5
    assert res["fallback_fraction"] < 0.25
