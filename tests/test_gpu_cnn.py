"""GPU parity of the corrector kernels (BF16 MFMA convolutions, backward passes,
Adam, coarse-graining) against the CPU reference in oracle/conv_ref.py.

The GPU rounds inputs, weights and hidden activations to bfloat16 and accumulates
in FP32; the reference is evaluated on the same bfloat16-rounded inputs and
weights, with its hidden activations rounded to bfloat16 at the same places, so
the remaining difference is the FP32 accumulation order (plus an occasional
activation that rounds to the neighbouring bfloat16 value).  Tolerances follow
2^-8 sqrt(K) relative per element, about 1e-2."""
import numpy as np
import pytest

from gpu_helpers import rel_l2
from oracle import conv_ref
from paper_2411_18341_amd import phx

pytestmark = pytest.mark.gpu


def ref_forward_bf16(layers, x):
    """Reference forward with bfloat16 rounding where the GPU rounds."""
    h = conv_ref.to_bf16(x)
    for k, (w, b) in enumerate(layers):
        h = conv_ref.conv3x3(h, conv_ref.to_bf16(w), b)
        if k < 3:
            h = conv_ref.to_bf16(conv_ref.relu(h))
    return h


def make(batch, H=32, W=64, seed=0):
    import torch
    net = phx.Corrector(H, W, batch)
    net.init_random(seed, scale=1.0)
    rng = np.random.default_rng(seed + 1)
    x = rng.standard_normal((batch, H, W, 4)).astype(np.float32)
    t = rng.standard_normal((batch, H, W, 3)).astype(np.float32) * 0.1
    return net, x, t, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()


def test_forward_parity():
    net, x, t, xd, td = make(3)
    layers = [(conv_ref.to_bf16(w), b) for w, b in net.get_weights()]
    y = net.forward(xd).cpu().numpy()
    ref = ref_forward_bf16(layers, x.transpose(0, 3, 1, 2)).transpose(0, 2, 3, 1)
    e = rel_l2(y, ref)
    print(f"forward rel L2 {e:.2e}")
    assert e < 1e-2
    assert np.max(np.abs(y - ref)) < 2.0 ** -6 * np.max(np.abs(ref))
    net.close()


@pytest.mark.parametrize("H,W", [(20, 64), (5, 32), (1, 96)])
def test_forward_parity_ragged_height(H, W):
    """Heights that are not a multiple of the forward kernel's tile height (the last
    tile's missing rows wrap circularly when staged and are not stored), down to a
    single row whose vertical neighbours are itself."""
    net, x, t, xd, td = make(3, H=H, W=W, seed=13)
    layers = [(conv_ref.to_bf16(w), b) for w, b in net.get_weights()]
    y = net.forward(xd).cpu().numpy()
    ref = ref_forward_bf16(layers, x.transpose(0, 3, 1, 2)).transpose(0, 2, 3, 1)
    e = rel_l2(y, ref)
    print(f"{H} x {W} forward rel L2 {e:.2e}")
    assert e < 1e-2
    assert np.max(np.abs(y - ref)) < 2.0 ** -6 * np.max(np.abs(ref))
    net.close()


def test_forward_input_paths_agree():
    """The first layer reads 16-byte-aligned float32 features itself and packs other
    inputs to bfloat16 first; training packs them too.  All give the same bits."""
    import torch
    net, x, t, xd, td = make(2, seed=17)
    y0 = net.forward(xd).clone()
    buf = torch.empty(xd.numel() + 1, dtype=torch.float32, device="cuda")
    xu = buf[1:].view(xd.shape)
    xu.copy_(xd)
    assert xu.data_ptr() % 16 != 0
    y1 = net.forward(xu)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    net.close()


def test_inference_pass_matches_training_forward():
    """Inference runs layers 1 and 2 as one fused kernel; training runs the layers one
    by one.  Both accumulate every output in the same order, so their outputs are the
    same bits: the loss that gradients() forms from its own forward pass equals the
    loss of forward()'s output up to the order of the (exact) double-precision sum."""
    import torch
    net, x, t, xd, td = make(4, H=44, W=96, seed=23)
    y = net.forward(xd).cpu().numpy()
    net.gradients(xd, td)
    torch.cuda.synchronize()
    d = (y - t).astype(np.float64)  # float32 differences, as the loss kernel forms them
    ref = float(np.sum(d * d) / d.size)
    print(f"loss {net.loss.item():.17g} vs {ref:.17g}")
    assert abs(net.loss.item() - ref) <= 1e-12 * ref
    net.close()


def test_gradients_parity():
    net, x, t, xd, td = make(2, seed=3)
    layers = [(conv_ref.to_bf16(w), b) for w, b in net.get_weights()]
    g = net.gradients(xd, td)
    import torch
    torch.cuda.synchronize()
    got = net.unpack(g.cpu().numpy())
    loss_ref, grads_ref = conv_ref.loss_and_grads(layers, conv_ref.to_bf16(x.transpose(0, 3, 1, 2)),
                                                  t.transpose(0, 3, 1, 2))
    assert abs(net.loss.item() - loss_ref) < 1e-2 * loss_ref
    for l in range(4):
        ew = rel_l2(got[l][0], grads_ref[l][0])
        eb = rel_l2(got[l][1], grads_ref[l][1])
        print(f"layer {l}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        assert ew < 3e-2 and eb < 3e-2
    # padded entries of the gradient stay exactly zero
    flat = g.cpu().numpy()
    repacked = np.zeros_like(flat)
    net2 = net
    tmp = net2.params.clone()
    net2.set_weights(got)
    repacked = net2.params.cpu().numpy()
    net2.params.copy_(tmp)
    mask = repacked != 0
    assert np.all(flat[~mask] == 0)
    net.close()


def test_forward_and_gradients_parity_256_batch16():
    """The workload's size: 16 images of 256 x 256, so that the persistent forward and
    weight-gradient kernels walk many tiles per workgroup and sum partials from many
    workgroups.  Forward output, loss and every layer's weight and bias gradient
    against the reference on the same bfloat16-rounded inputs and weights."""
    import torch
    net, x, t, xd, td = make(16, H=256, W=256, seed=21)
    layers = [(conv_ref.to_bf16(w), b) for w, b in net.get_weights()]
    y = net.forward(xd).cpu().numpy()
    xr = x.transpose(0, 3, 1, 2)
    ref = ref_forward_bf16(layers, xr).transpose(0, 2, 3, 1)
    e = rel_l2(y, ref)
    print(f"256^2 x 16 forward rel L2 {e:.2e}")
    assert e < 1e-2
    assert np.max(np.abs(y - ref)) < 2.0 ** -6 * np.max(np.abs(ref))
    g = net.gradients(xd, td)
    torch.cuda.synchronize()
    got = net.unpack(g.cpu().numpy())
    loss_ref, grads_ref = conv_ref.loss_and_grads(layers, conv_ref.to_bf16(xr), t.transpose(0, 3, 1, 2))
    assert abs(net.loss.item() - loss_ref) < 1e-2 * loss_ref
    for l in range(4):
        ew = rel_l2(got[l][0], grads_ref[l][0])
        eb = rel_l2(got[l][1], grads_ref[l][1])
        print(f"256^2 x 16 layer {l}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        assert ew < 3e-2 and eb < 3e-2
    net.close()


def test_adam_parity():
    net, x, t, xd, td = make(2, seed=5)
    import torch
    p0 = net.params.cpu().numpy().astype(np.float64)
    g = net.gradients(xd, td).clone()
    net.adam(lr=1e-3, grads=g)
    g2 = net.gradients(xd, td).clone()
    net.adam(lr=1e-3, grads=g2)
    torch.cuda.synchronize()
    th, m, v = conv_ref.adam_step(p0, g.cpu().numpy().astype(np.float64), 0, 0, 1)
    th, m, v = conv_ref.adam_step(th, g2.cpu().numpy().astype(np.float64), m, v, 2)
    got = net.params.cpu().numpy()
    assert np.max(np.abs(got - th)) < 1e-6
    net.close()


def test_training_reduces_loss():
    """Fit a fixed random target network: the loss falls by a large factor."""
    import torch
    net, x, t, xd, td = make(4, seed=7)
    teacher = phx.Corrector(32, 64, 4)
    teacher.init_random(99, scale=1.0)
    tgt = teacher.forward(xd).clone()
    l0 = None
    tail = []
    for it in range(300):
        net.train_step(xd, tgt, lr=2e-3)
        if it == 0:
            torch.cuda.synchronize()
            l0 = net.loss.item()
        if it >= 280:
            tail.append(net.loss.item())
    # the loss of single Adam steps fluctuates: judge the mean of the last 20
    l1 = sum(tail) / len(tail)
    print(f"loss {l0:.3e} -> {l1:.3e} (mean of the last 20 steps)")
    assert l1 < 0.25 * l0
    net.close()
    teacher.close()


@pytest.mark.parametrize("precision", [phx.PHX_C64, phx.PHX_C128])
def test_coarsen_features_residual_apply(precision):
    import torch
    cdt, rdt = phx.torch_dtypes(precision)
    rng = np.random.default_rng(11)
    psi = rng.standard_normal((64, 96)) + 1j * rng.standard_normal((64, 96))
    n = rng.uniform(0, 5, (64, 96))
    P = rng.uniform(0, 3, (64, 96))
    d = lambda a, t: torch.from_numpy(a).to("cuda", t).contiguous()
    psi_d, n_d, P_d = d(psi, cdt), d(n, rdt), d(P, rdt)
    pc = torch.empty((16, 24), dtype=cdt, device="cuda")
    nc = torch.empty((16, 24), dtype=rdt, device="cuda")
    Pc = torch.empty((16, 24), dtype=rdt, device="cuda")
    phx.phx_coarsen(precision, psi_d, n_d, P_d, 96, 64, 4, pc, nc, Pc)
    tol = 1e-6 if precision == phx.PHX_C64 else 1e-13
    q = lambda a: np.asarray(a, np.complex128 if np.iscomplexobj(a) else np.float64)
    psi_q = psi_d.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(pc.cpu().numpy() - conv_ref.block_mean(psi_q))) < tol * 4
    assert np.max(np.abs(nc.cpu().numpy() - conv_ref.block_mean(n_d.cpu().numpy().astype(np.float64)))) < tol * 10
    x = torch.empty((16, 24, 4), dtype=torch.float32, device="cuda")
    phx.phx_corrector_features(precision, pc, nc, Pc, 24, 16, 2.0, 5.0, 3.0, x)
    xs = x.cpu().numpy()
    pcn = pc.cpu().numpy()
    assert np.allclose(xs[..., 0], pcn.real / 2.0, rtol=1e-6, atol=1e-7)
    assert np.allclose(xs[..., 1], pcn.imag / 2.0, rtol=1e-6, atol=1e-7)
    assert np.allclose(xs[..., 2], nc.cpu().numpy() / 5.0, rtol=1e-6)
    assert np.allclose(xs[..., 3], Pc.cpu().numpy() / 3.0, rtol=1e-6)
    r = torch.empty((16, 24, 3), dtype=torch.float32, device="cuda")
    pref = pc * 1.5
    nref = nc + 1.0
    phx.phx_corrector_residual(precision, pref, nref, pc, nc, 24, 16, 2.0, 5.0, r)
    rs = r.cpu().numpy()
    assert np.allclose(rs[..., 0], (0.5 * pcn.real) / 2.0, rtol=1e-5, atol=1e-7)
    assert np.allclose(rs[..., 2], 1.0 / 5.0, rtol=1e-5)
    # applying the residual restores the reference
    phx.phx_corrector_apply(precision, pc, nc, r, 24, 16, 2.0, 5.0)
    assert np.allclose(pc.cpu().numpy(), pref.cpu().numpy(), rtol=1e-5, atol=1e-6)
    assert np.allclose(nc.cpu().numpy(), nref.cpu().numpy(), rtol=1e-5)
