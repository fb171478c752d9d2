"""xf_rhs_noalloc, the right-hand side for callers that cannot allocate:
through the C ABI, against xf_rhs on the same inputs (bit for bit: the same
kernels on the same data), on two calls in a row with the second on a smaller
grid (the static scratch keeps the first call's contents), and the rejection
of a problem whose workspace exceeds the static buffer."""
import numpy as np
import pytest

from paper_2403_05910_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _xf():
    from paper_2403_05910_amd import xf
    return xf


def _noalloc(xf, ctx, U, out):
    xf.xf_rhs_noalloc(ctx.handle, ctx._ptr(U), ctx._ptr(out), ctx._stream())
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_rhs_on_two_calls(precision):
    xf = _xf()
    tab = W.sampled_table(W.W9, 0)
    big = W.random_smooth_state(tab, (40, 36, 30), seed=3, jump=True, bc=(1, 1, 0, 0, 0, 0))
    small = W.random_smooth_state(tab, (12, 9, 7), seed=4, jump=True)
    for case in (big, small):
        print(f"[noalloc] {precision} grid {case.n}", flush=True)
        ctx = xf.Context.from_case(case, precision)
        assert xf.xf_workspace_bytes(ctx.handle, xf.XF_OP_RHS) <= xf.XF_NOALLOC_BYTES
        U = ctx.state_from_numpy(case.U)
        ctx.fill_ghosts(U)
        ref = ctx.rhs(U)
        out = torch.full_like(ref, np.nan)
        _noalloc(xf, ctx, U, out)
        torch.cuda.synchronize()
        assert ctx.status() == 0
        assert torch.equal(out, ref)
        # a second call on the same context, into a fresh buffer
        out2 = torch.full_like(ref, np.nan)
        _noalloc(xf, ctx, U, out2)
        assert torch.equal(out2, ref)
        ctx.close()


def test_noalloc_rejects_problems_beyond_the_static_buffer():
    xf = _xf()
    tab = W.sampled_table([2.0, 28.0], 0)
    ctx = xf.Context((160, 160, 160), (1.0 / 160,) * 3, (0,) * 6, tab.W, tab.a, tab.T_lo, tab.T_hi)
    assert xf.xf_workspace_bytes(ctx.handle, xf.XF_OP_RHS) > xf.XF_NOALLOC_BYTES
    U = ctx.new_state()
    out = ctx.new_state()
    with pytest.raises(xf.XfError) as e:
        _noalloc(xf, ctx, U, out)
    assert e.value.code == xf.XF_ETOOLARGE
    with pytest.raises(xf.XfError) as e:
        xf.xf_rhs_noalloc(ctx.handle, ctx._ptr(U), ctx._ptr(U), ctx._stream())
    assert e.value.code == xf.XF_EINVAL
    ctx.close()
