"""The allocation-free entry point (triot_apply_noalloc) against triot_apply
with a caller workspace, through the C ABI: the reductions that need a
workspace (moments with the covariance, the inner product, a marginal whose
parts are combined through the scratch, the bounding box) and one
element-wise op, each on two calls in a row, the second with a smaller
input.  Results must equal triot_apply's bit for bit (same kernels, same
launch), and the moments stay within 1e-6 of the float64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _both(op, tensors, shapes, counter, params_ws, params_na, out_ws, out_na):
    """Run op through triot_apply (fresh caller workspace) and through
    triot_apply_noalloc; both statuses must be OK."""
    d = len(shapes[0])
    ptrs = [t.data_ptr() for t in tensors]
    nbytes = L.triot_workspace_size(op, len(shapes), d, shapes, counter)
    assert nbytes <= L.NOALLOC_SCRATCH_BYTES
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
    st = L.triot_apply(op, len(tensors), d, shapes, counter, ptrs, None, params_ws,
                       out_ws.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    assert st == L.OK, L.status_string(st)
    st = L.triot_apply_noalloc(op, len(tensors), d, shapes, counter, ptrs, None, params_na,
                               out_na.data_ptr(), _stream())
    assert st == L.OK, L.status_string(st)
    torch.cuda.synchronize()


def _bits_equal(a, b):
    return a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()


@pytest.mark.parametrize("shapes", [[(16,) * 6, (9, 7, 5)], [(64, 48, 40), (3, 2)]])
def test_noalloc_moments_two_calls(shapes):
    for k, shape in enumerate(shapes):
        announce("noalloc moments", k, shape)
        p_np = inputs.cfg3_values(shape)
        p = torch.from_numpy(p_np).cuda()
        d = len(shape)
        nout = 1 + d + d * (d + 1) // 2
        o32a = torch.full((nout,), -1.0, device="cuda")
        o64a = torch.full((nout,), -1.0, dtype=torch.float64, device="cuda")
        o32b = torch.full((nout,), -2.0, device="cuda")
        o64b = torch.full((nout,), -2.0, dtype=torch.float64, device="cuda")
        flags = L.MOMENTS_FIRST | L.MOMENTS_COV
        _both(L.OP_MOMENTS, [p], [shape], None, L.MomentsParams(flags, o64a.data_ptr()),
              L.MomentsParams(flags, o64b.data_ptr()), o32a, o32b)
        assert _bits_equal(o32a, o32b) and _bits_equal(o64a, o64b)
        # within 1e-6 relative of the float64 oracle; an entry whose exact
        # value is 0 within 1e-6 of the covariance diagonal's scale
        ref = oracle.moments(shape, [p_np.reshape(-1)], [shape], cov=True)[:nout]
        got = o32b.cpu().numpy().astype(np.float64)
        diag = max(abs(ref[1 + d + i * d - i * (i - 1) // 2]) for i in range(d))
        absok = np.abs(got - ref) <= 1e-6 * 1e-6 * max(1.0, diag)
        with np.errstate(divide="ignore", invalid="ignore"):
            rel = np.abs(got - ref) / np.abs(ref)
        assert ((rel <= 1e-6) | absok).all(), (shape, rel)


def test_noalloc_dot_marginal_bbox_two_calls():
    for k, shape in enumerate([(16,) * 6, (5, 6, 7)]):
        announce("noalloc dot/marginal/bbox", k, shape)
        g = np.random.default_rng(40 + k)
        a_np = g.random(shape, dtype=np.float32)
        b_np = np.where(g.random(shape) < 0.01, g.random(shape), 0).astype(np.float32)
        a = torch.from_numpy(a_np).cuda()
        b = torch.from_numpy(b_np).cuda()
        sh = [shape, shape]
        # inner product
        oa, ob = torch.empty(1, device="cuda"), torch.empty(1, device="cuda")
        ea = torch.empty(1, dtype=torch.float64, device="cuda")
        eb = torch.empty(1, dtype=torch.float64, device="cuda")
        _both(L.OP_DOT, [a, b], sh, None, L.ReduceParams(ea.data_ptr()),
              L.ReduceParams(eb.data_ptr()), oa, ob)
        assert _bits_equal(oa, ob) and _bits_equal(ea, eb)
        want = oracle.dot(shape, [a_np.reshape(-1), b_np.reshape(-1)], sh)
        assert abs(eb.item() - want) <= 1e-10 * max(1.0, abs(want))
        # marginal keeping axis 0 (few outputs: the parts meet in the scratch)
        keep = 1
        kshape = (shape[0],)
        ma, mb = torch.empty(kshape, device="cuda"), torch.empty(kshape, device="cuda")
        m64a = torch.empty(kshape, dtype=torch.float64, device="cuda")
        m64b = torch.empty(kshape, dtype=torch.float64, device="cuda")
        _both(L.OP_MARGINAL, [a], [shape], None, L.MarginalParams(keep, m64a.data_ptr()),
              L.MarginalParams(keep, m64b.data_ptr()), ma, mb)
        assert _bits_equal(ma, mb) and _bits_equal(m64a, m64b)
        wantm = oracle.marginal(shape, [True] + [False] * (len(shape) - 1),
                                [a_np.reshape(-1)], [shape])
        assert np.allclose(m64b.cpu().numpy().reshape(-1), np.asarray(wantm).reshape(-1),
                           rtol=1e-9, atol=0)
        # nonzero bounding box
        d = len(shape)
        xa = torch.empty(2 * d, dtype=torch.int64, device="cuda")
        xb = torch.empty(2 * d, dtype=torch.int64, device="cuda")
        _both(L.OP_BBOX, [a, b], sh, None, None, None, xa, xb)
        assert torch.equal(xa, xb)
        wantb = oracle.bbox(shape, [a_np.reshape(-1), b_np.reshape(-1)], sh)
        assert np.array_equal(xb.cpu().numpy().reshape(-1), np.asarray(wantb).reshape(-1))


def test_noalloc_elementwise_two_calls():
    for k, (src_s, dst_s) in enumerate([((48, 40, 36), (64, 64, 64)), ((5, 3), (7, 9))]):
        announce("noalloc copy", k, src_s, dst_s)
        src = torch.from_numpy(inputs.uniform(1, src_s, 70, k)).cuda()
        da = torch.zeros(dst_s, device="cuda")
        db = torch.zeros(dst_s, device="cuda")
        ptrs_a, ptrs_b = [da.data_ptr(), src.data_ptr()], [db.data_ptr(), src.data_ptr()]
        st = L.triot_apply(L.OP_COPY, 2, len(src_s), [dst_s, src_s], src_s, ptrs_a, None,
                           L.CopyParams(4), 0, 0, 0, _stream())
        assert st == L.OK
        st = L.triot_apply_noalloc(L.OP_COPY, 2, len(src_s), [dst_s, src_s], src_s, ptrs_b, None,
                                   L.CopyParams(4), 0, _stream())
        assert st == L.OK
        torch.cuda.synchronize()
        assert _bits_equal(da, db)
        want = np.zeros(dst_s, dtype=np.float32)
        oracle.copy(src_s, want.reshape(-1), dst_s, src.cpu().numpy().reshape(-1), src_s)
        assert db.cpu().numpy().tobytes() == want.tobytes()


def test_noalloc_errors_enqueue_nothing():
    announce("noalloc errors")
    a = torch.full((4, 4), 3.0, device="cuda")
    b = torch.zeros((3, 5), device="cuda")
    st = L.triot_apply_noalloc(L.OP_COPY, 2, 2, [(4, 4), (3, 5)], (4, 4),
                               [a.data_ptr(), b.data_ptr()], None, L.CopyParams(4), 0, _stream())
    assert st == L.E_BOUNDS
    st = L.triot_apply_noalloc(L.OP_MOMENTS, 1, 2, [(4, 4)], None, [a.data_ptr()], None,
                               L.MomentsParams(L.MOMENTS_FIRST, 0), 0, _stream())
    assert st == L.E_INVALID          # moments need an out pointer
    torch.cuda.synchronize()
    assert bool((a == 3.0).all())
