"""GPU: the surrogate network's kernels (through the C ABI) against the FP64 CPU
oracle on the same BF16-valued weights and inputs.

Bars: forward output, parameter gradients (per layer) and input gradients
within rel-L2 1e-2 of the FP64 oracle (the kernels round activations and
gradients to BF16 before every product); Adam within 1e-5 of the oracle's
recursion; training reduces the loss of a teacher-student regression.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2609_01978_amd as P  # noqa: E402
from oracle import mlp_oracle as Q  # noqa: E402

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def bf16_round(a):
    """float32 values rounded to the nearest BF16 (ties to even), as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def make(seed, n_in, H, n_out, B, wscale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, H), (H, H), (H, n_out)):
        parts.append(rng.uniform(-1, 1, fi * fo) * wscale / np.sqrt(fi))
        parts.append(rng.uniform(-0.1, 0.1, fo))
    theta = bf16_round(np.concatenate(parts).astype(np.float32))
    x = bf16_round(rng.uniform(-1, 1, (B, n_in)).astype(np.float32))
    t = rng.standard_normal((B, n_out)).astype(np.float32)
    return theta, x, t


def groups(v, n_in, H, n_out):
    return Q.unpack(np.asarray(v, dtype=np.float64), n_in, H, n_out)


@pytest.mark.parametrize("n_in,H,n_out,B", [(33, 96, 300, 37), (33, 512, 16384, 64), (5, 40, 70, 1)])
def test_forward_backward_vs_oracle(n_in, H, n_out, B):
    print(f"[gpu-mlp] dims {n_in}/{H}/{n_out} batch {B}", flush=True)
    theta, x, t = make(1, n_in, H, n_out, B)
    m = P.MLP(n_in, H, n_out, max(B, 8))
    assert m.n_params == Q.param_count(n_in, H, n_out)
    m.set_params(torch.from_numpy(theta).cuda())
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = m.forward(xd)
    loss, g, dx, y2 = m.backward(xd, td)
    torch.cuda.synchronize()
    yo, _ = Q.forward(theta.astype(np.float64), x, n_in, H, n_out)
    Lo, go, dxo = Q.backward(theta.astype(np.float64), x, t, n_in, H, n_out)
    assert rel_l2(y.cpu().numpy(), yo) <= 1e-2
    assert torch.equal(y, y2)
    assert abs(float(loss.item()) / Lo - 1) <= 1e-2
    for k, (a, b) in enumerate(zip(groups(g.cpu().numpy(), n_in, H, n_out), groups(go, n_in, H, n_out))):
        e = rel_l2(a, b)
        print(f"[gpu-mlp]   grad group {k} rel-L2 {e:.2e}", flush=True)
        assert e <= 1e-2, k
    assert rel_l2(dx.cpu().numpy(), dxo) <= 1e-2
    # parameters read back unchanged
    assert torch.equal(m.get_params().cpu(), torch.from_numpy(theta))


def test_adam_vs_oracle():
    n_in, H, n_out = 7, 24, 50
    theta, _, _ = make(2, n_in, H, n_out, 1)
    m = P.MLP(n_in, H, n_out, 4)
    m.set_params(torch.from_numpy(theta).cuda())
    rng = np.random.default_rng(3)
    th, mo, vo = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in range(1, 4):
        g = (rng.standard_normal(theta.size) * 10.0 ** rng.uniform(-4, 1, theta.size)).astype(np.float32)
        m.adam_update(torch.from_numpy(g).cuda(), 1e-3)
        th, mo, vo = Q.adam_step(th, g.astype(np.float64), mo, vo, step, 1e-3)
    got = m.get_params().cpu().numpy().astype(np.float64)
    assert rel_l2(got - theta, th - theta) <= 1e-5


def test_training_reduces_loss():
    """Student learns a random teacher of the same shape (regression)."""
    n_in, H, n_out, B = 33, 128, 256, 64
    teacher, _, _ = make(5, n_in, H, n_out, 1, wscale=2.0)
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (1024, n_in)).astype(np.float32)
    T, _ = Q.forward(teacher.astype(np.float64), X, n_in, H, n_out)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T.astype(np.float32)).cuda()
    student, _, _ = make(7, n_in, H, n_out, 1)
    m = P.MLP(n_in, H, n_out, B)
    m.set_params(torch.from_numpy(student).cuda())
    first = None
    for ep in range(40):
        tot = 0.0
        for s in range(0, 1024, B):
            tot += float(m.train_step(Xd[s:s + B], Td[s:s + B], 3e-3).item())
        if first is None:
            first = tot
    print(f"[gpu-mlp] training loss {first:.4f} -> {tot:.4f}", flush=True)
    assert tot < 0.1 * first


def test_log_intensity_roundtrip():
    rng = np.random.default_rng(8)
    U = (rng.standard_normal(5000) + 1j * rng.standard_normal(5000)) * 30.0
    roi = torch.from_numpy(np.stack([U.real, U.imag], axis=1).ravel()).cuda()
    out = torch.empty(5000, dtype=torch.float32, device="cuda")
    P.log_intensity(roi, 5000, 900.0, 1e-6, out)
    torch.cuda.synchronize()
    want = np.log(np.abs(U) ** 2 / 900.0 + 1e-6)
    assert np.allclose(out.cpu().numpy(), want, rtol=1e-6, atol=1e-6)
    back = torch.empty(10000, dtype=torch.float64, device="cuda")
    P.field_from_log_intensity(out, 5000, 900.0, 1e-6, back)
    torch.cuda.synchronize()
    b = back.cpu().numpy().reshape(-1, 2)
    assert np.all(b[:, 1] == 0.0)
    assert np.allclose(b[:, 0] ** 2, np.abs(U) ** 2, rtol=1e-5, atol=1e-3)
