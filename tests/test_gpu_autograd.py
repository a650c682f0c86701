"""The differentiable pipeline at full size: pad (24,)^5 -> (32,)^5, product
with a (28,30,32,26,32) weight over the intersection, E-based loss, forward
and backward through torch.autograd with the library's adjoint kernels.

The gradient is checked against the oracle's float64 analytic gradient
(element by element) and against float64 central finite differences of the
oracle pipeline (random unit directions and single coordinates), at relative
error 1e-4."""
import numpy as np
import pytest
import torch

from oracle import pipeline
from paper_1608_00099_amd import api, autograd, inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _gpu_grad(x_np, w_np, lam):
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    w = torch.from_numpy(w_np).cuda().requires_grad_(True)
    lam_t = torch.from_numpy(lam.astype(np.float32)).cuda()
    P = autograd.pad_embed(x, inputs.CFG5_P)
    y = autograd.mul(P, w)
    M, E, C = autograd.moments(y)
    loss = (lam_t * E).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (float(loss), x.grad.cpu().numpy().astype(np.float64).reshape(-1),
            w.grad.cpu().numpy().astype(np.float64).reshape(-1))


@pytest.mark.timeout(900)
def test_pipeline_gradient_full_size():
    announce("autograd cfg5")
    x_np, w_np, lam = inputs.cfg5_values()
    xs, ps, ws = inputs.CFG5_X, inputs.CFG5_P, inputs.CFG5_W
    loss, gx, gw = _gpu_grad(x_np, w_np, lam)
    x64 = x_np.astype(np.float64).reshape(-1)
    w64 = w_np.astype(np.float64).reshape(-1)
    L_ref = pipeline.loss(x64, w64, lam, xs, ps, ws)
    assert abs(loss - L_ref) <= 1e-6 * max(1.0, abs(L_ref))
    rx, rw = pipeline.gradient(x64, w64, lam, xs, ps, ws)
    for g, r in ((gx, rx), (gw, rw)):
        assert np.linalg.norm(g - r) <= 1e-4 * np.linalg.norm(r)
        den = np.maximum(np.abs(r), 1e-3 * np.sqrt(np.mean(r * r)))
        assert (np.abs(g - r) / den).max() <= 1e-4
    # float64 central differences of the oracle pipeline
    rng = np.random.default_rng(55)
    for which, vec, grad in ((0, x64, gx), (1, w64, gw)):
        for _ in range(3):
            v = rng.standard_normal(vec.size)
            v /= np.linalg.norm(v)
            # The loss is a ratio of sums linear in x and w, so the central
            # difference's truncation error is ~ h * |dM/dv| / M ~ 1e-7 h;
            # a large step keeps the float64 summation noise of the two
            # 22M-term loss evaluations (~1e-11 absolute) far below 1e-4.
            h = 1.0
            a = [x64, w64]
            b = [x64, w64]
            a[which] = vec + h * v
            b[which] = vec - h * v
            fd = (pipeline.loss(a[0], a[1], lam, xs, ps, ws) -
                  pipeline.loss(b[0], b[1], lam, xs, ps, ws)) / (2 * h)
            assert abs(float(np.dot(grad, v)) - fd) <= 1e-4 * abs(fd)
        for k in rng.choice(vec.size, size=3, replace=False):
            h = 0.25
            a = [x64, w64]
            b = [x64, w64]
            a[which] = vec.copy()
            b[which] = vec.copy()
            a[which][k] += h
            b[which][k] -= h
            fd = (pipeline.loss(a[0], a[1], lam, xs, ps, ws) -
                  pipeline.loss(b[0], b[1], lam, xs, ps, ws)) / (2 * h)
            assert abs(grad[k] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.sqrt(np.mean(grad ** 2)))


def test_autograd_functions_match_raw_kernels():
    announce("autograd vs raw")
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.random((5, 6, 7), dtype=np.float32)).cuda().requires_grad_(True)
    P = autograd.pad_embed(x, (8, 9, 10))
    gP = torch.from_numpy(rng.standard_normal((8, 9, 10)).astype(np.float32)).cuda()
    P.backward(gP)
    assert torch.equal(x.grad, api.crop(gP, (5, 6, 7)))
    # moments with the covariance: backward equals the adjoint kernel
    p = torch.from_numpy(rng.random((6, 5, 4), dtype=np.float32)).cuda().requires_grad_(True)
    M, E, C = autograd.Moments.apply(p, True)
    gE = torch.from_numpy(rng.standard_normal(3).astype(np.float32)).cuda()
    gC = torch.from_numpy(rng.standard_normal(6).astype(np.float32)).cuda()
    (E * gE).sum().add_((C * gC).sum()).backward()
    o32, o64 = api.moments(p.detach(), cov=True)
    gm = torch.cat([torch.zeros(1, device="cuda"), gE, gC])
    g = api.moments_adj(p.shape, o64, gm, cov=True)
    assert torch.allclose(p.grad, g, rtol=1e-6, atol=0)


def test_pipeline_in_captured_graphs_matches_eager():
    """Forward and backward of the pipeline captured as graphs
    (torch.cuda.make_graphed_callables over the library's Functions) and
    replayed, with eager work and synchronisation between replays: every
    replay gives the eager loss and gradients bit for bit."""
    announce("autograd cfg5 graphed")
    x_np, w_np, lam = inputs.cfg5_values()
    lam_t = torch.from_numpy(lam.astype(np.float32)).cuda()

    def step(x, w):
        P = autograd.pad_embed(x, inputs.CFG5_P)
        y = autograd.mul(P, w)
        M, E, C = autograd.moments(y)
        return (lam_t * E).sum()

    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    w = torch.from_numpy(w_np).cuda().requires_grad_(True)
    loss = step(x, w)
    loss.backward()
    torch.cuda.synchronize()
    ref = (loss.detach().cpu().numpy(), x.grad.cpu().numpy(), w.grad.cpu().numpy())
    xg = x.detach().clone().requires_grad_(True)
    wg = w.detach().clone().requires_grad_(True)
    g_step = torch.cuda.make_graphed_callables(step, (xg, wg))
    for rep in range(3):
        xg.grad = None
        wg.grad = None
        other = torch.arange(4096, device="cuda", dtype=torch.float32)
        assert float(other.sum()) == 4096 * 4095 / 2           # eager work, synchronised
        loss = g_step(xg, wg)
        loss.backward()
        torch.cuda.synchronize()
        got = (loss.detach().cpu().numpy(), xg.grad.cpu().numpy(), wg.grad.cpu().numpy())
        for a, b in zip(got, ref):
            assert a.tobytes() == b.tobytes(), rep


def test_pipeline_captured_as_one_graph_matches_eager():
    """Forward and backward of the pipeline captured as ONE graph over the
    leaf tensors (autograd.CapturedStep) and replayed, with eager work,
    in-place input updates and synchronisation between replays: every
    replay gives the eager loss and gradients bit for bit."""
    announce("autograd cfg5 one captured step")
    x_np, w_np, lam = inputs.cfg5_values()
    lam_t = torch.from_numpy(lam.astype(np.float32)).cuda()

    def step(x, w):
        P = autograd.pad_embed(x, inputs.CFG5_P)
        y = autograd.mul(P, w)
        M, E, C = autograd.moments(y)
        return (lam_t * E).sum()

    def eager(xv, wv):
        x = torch.from_numpy(xv).cuda().requires_grad_(True)
        w = torch.from_numpy(wv).cuda().requires_grad_(True)
        loss = step(x, w)
        loss.backward()
        torch.cuda.synchronize()
        return loss.detach().cpu().numpy(), x.grad.cpu().numpy(), w.grad.cpu().numpy()

    xg = torch.from_numpy(x_np).cuda().requires_grad_(True)
    wg = torch.from_numpy(w_np).cuda().requires_grad_(True)
    cap = autograd.CapturedStep(step, (xg, wg))
    for rep in range(3):
        xv = (x_np * (1.0 + 0.25 * rep)).astype(np.float32)   # new values, written in place
        with torch.no_grad():
            xg.copy_(torch.from_numpy(xv))
        other = torch.arange(4096, device="cuda", dtype=torch.float32)
        assert float(other.sum()) == 4096 * 4095 / 2           # eager work, synchronised
        loss = cap.replay()
        torch.cuda.synchronize()
        got = (loss.detach().cpu().numpy(), xg.grad.cpu().numpy(), wg.grad.cpu().numpy())
        ref = eager(xv, w_np)
        for a, b in zip(got, ref):
            assert a.tobytes() == b.tobytes(), rep


def test_moments_backward_unused_outputs():
    """Only E used, only M used, and E and C used: the gradient equals the
    adjoint kernel on the partials with zeros where an output is unused."""
    announce("moments backward partial use")
    rng = np.random.default_rng(17)
    shape = (5, 6, 7)
    pn = rng.random(shape).astype(np.float32)
    for use in ("E", "M", "EC"):
        p = torch.from_numpy(pn).cuda().requires_grad_(True)
        cov = "C" in use
        M, E, C = autograd.moments(p, cov=cov)
        loss = 0.0
        if "M" in use:
            loss = loss + 3.0 * M.sum()
        if "E" in use:
            loss = loss + (torch.arange(1, 4, device="cuda", dtype=torch.float32) * E).sum()
        if "C" in use:
            loss = loss + (0.5 * C).sum()
        loss.backward()
        o32, o64 = api.moments(p.detach(), cov=cov)
        n = 1 + 3 + (6 if cov else 0)
        gm = torch.zeros(n, device="cuda")
        if "M" in use:
            gm[0] = 3.0
        if "E" in use:
            gm[1:4] = torch.arange(1, 4, device="cuda", dtype=torch.float32)
        if "C" in use:
            gm[4:] = 0.5
        g = api.moments_adj(shape, o64, gm, cov=cov)
        assert torch.equal(p.grad, g), use
