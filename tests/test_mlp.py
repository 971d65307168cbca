"""The ladder network: the FP64 reference is pinned by finite differences, and the
library's FP32 MFMA kernels agree with it (GPU)."""
import numpy as np
import pytest

from oracle import mlp


def random_problem(B, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, size=mlp.N_PARAMS)
    x = rng.normal(0, 1.0, size=(B, 32))
    q = rng.random((B, 64)) ** 3
    q /= q.sum(axis=1, keepdims=True)
    return p, x, q


@pytest.mark.parametrize("kind", ["softmax", "sigmoid"])
def test_reference_gradient_matches_finite_differences(kind):
    p, x, q = random_problem(5, seed=1)
    _, g = mlp.loss_grad(p, x, q, kind)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, size=300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, q, kind) - mlp.loss(p - e, x, q, kind)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_reference_sigmoid_loss_minimum():
    """The logistic cross entropy is minimised by s(z) = q: its value there is the
    binary entropy of q."""
    from oracle import mlp as M
    q = np.array([[0.2, 0.7, 0.5] + [0.5] * 61])
    ent = float(-(q * np.log(q) + (1 - q) * np.log(1 - q)).sum())
    parts = M.unpack(np.zeros(M.N_PARAMS))
    parts[5][:] = np.log(q[0] / (1 - q[0]))
    p = M.pack(parts)
    assert abs(M.loss(p, np.zeros((1, 32)), q, "sigmoid") - ent) < 1e-12


def test_reference_loss_bounds_and_zero_output_layer():
    """Cross entropy >= entropy of q, with equality iff softmax(z) = q; zero output
    weights and biases give uniform softmax, i.e. the geometric ladder."""
    p, x, q = random_problem(7, seed=3)
    ent = float(-(q * np.log(q)).sum(axis=1).mean())
    assert mlp.loss(p, x, q) >= ent - 1e-12
    parts = mlp.unpack(p)
    parts[4][...] = 0
    parts[5][...] = 0
    z, _ = mlp.forward(mlp.pack(parts), x)
    assert np.allclose(mlp.softmax(z), 1 / 64)


def test_reference_adam_first_step_is_sign_step():
    g = np.array([0.5, -2.0, 1e-3])
    p1, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(p1, -0.1 * np.sign(g), atol=1e-6)


@pytest.fixture(scope="module")
def ptq():
    import torch
    from paper_1004_0023_amd import ptqmc
    torch.cuda.set_device(0)
    ptqmc.lib()
    return ptqmc


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["softmax", "sigmoid"])
@pytest.mark.parametrize("B", [1, 37, 256])
def test_gpu_forward_and_gradient_match_reference(ptq, B, kind):
    print(f"case: ladder network forward/backward, batch {B}, {kind} loss", flush=True)
    if kind == "sigmoid":
        q_rng = np.random.default_rng(B + 1000)
    p, x, q = random_problem(B, seed=B)
    net = ptq.LadderNet(p.astype(np.float32))
    z = net.forward(x.astype(np.float32)).cpu().numpy()
    pr = net.numpy_params().astype(np.float64)  # the FP32 parameters the kernels used
    z_ref, _ = mlp.forward(pr, x.astype(np.float32).astype(np.float64))
    assert np.allclose(z, z_ref, rtol=1e-4, atol=1e-4 * np.abs(z_ref).max())
    if kind == "sigmoid":
        q = q_rng.random((B, 64))
    code = ptq.MLP_LOSS_SOFTMAX if kind == "softmax" else ptq.MLP_LOSS_SIGMOID
    loss = net.loss_grad(x.astype(np.float32), q.astype(np.float32), code)
    g = net.grads.cpu().numpy().astype(np.float64)
    l_ref, g_ref = mlp.loss_grad(pr, x.astype(np.float32).astype(np.float64),
                                 q.astype(np.float32).astype(np.float64), kind)
    assert abs(loss - l_ref) <= 1e-4 * max(1.0, abs(l_ref))
    scale = np.abs(g_ref).max()
    assert np.allclose(g, g_ref, rtol=2e-3, atol=2e-4 * scale)


@pytest.mark.gpu
def test_gpu_adam_matches_reference(ptq):
    print("case: ladder network Adam step", flush=True)
    p, x, q = random_problem(64, seed=9)
    net = ptq.LadderNet(p.astype(np.float32))
    pr = net.numpy_params().astype(np.float64)
    m = np.zeros_like(pr)
    v = np.zeros_like(pr)
    for step in range(1, 4):
        net.loss_grad(x.astype(np.float32), q.astype(np.float32), ptq.MLP_LOSS_SOFTMAX)
        g = net.grads.cpu().numpy().astype(np.float64)
        net.adam(1e-3)
        pr, m, v = mlp.adam(pr, g, m, v, step, 1e-3)
        got = net.numpy_params().astype(np.float64)
        assert np.allclose(got, pr, rtol=1e-5, atol=1e-6)
        pr = got
