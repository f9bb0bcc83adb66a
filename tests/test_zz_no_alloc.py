"""fdtd_forward_noalloc: the forward entry point whose workspace is the library's own device array
(for callers that cannot allocate).  Its loss, loss series, final fields and store must equal
fdtd_forward's bit for bit, on two calls in a row, the second on a smaller problem (the array
keeps the first call's contents); its record must feed fdtd_backward (needs an MI355X)."""

from dataclasses import replace

import numpy as np
import pytest
import torch

import workloads as w
import paper_2603_24027_amd as pk

from gpu_helpers import require_gpu, say, store_layout

pytestmark = pytest.mark.gpu


def _problems():
    big = replace(w.ragged(steps=23), name="ragged_23_steps")   # odd 70x37x29 (75110 cells), plane source
    small = w.c1()                                              # 32^3 (32768 cells), PML 8, dipole
    return big, small


def _run(prob, dtype, k, noalloc):
    g = pk.Gradient(prob, dtype, k, series=True)
    eps = torch.from_numpy(np.ascontiguousarray(prob.eps, np.float32)).cuda()
    loss = (g.forward_noalloc if noalloc else g.forward)(eps)
    torch.cuda.synchronize()
    return g, float(loss.item())


@pytest.mark.parametrize("dtype,k", [("fp32", 1), ("fp8_e4m3_scaled", 3)])
def test_noalloc_forward_equals_forward_on_two_calls(dtype, k):
    require_gpu()
    big, small = _problems()
    assert big.cells > small.cells
    say("noalloc vs forward", dtype, "k", k)
    refs = [_run(p, dtype, k, False) for p in (big, small)]
    outs = [_run(p, dtype, k, True) for p in (big, small)]          # the second call reuses the array
    for (ref, lref), (got, lgot), p in zip(refs, outs, (big, small)):
        say("  %s: loss %.9e (forward %.9e)" % (p.name, lgot, lref))
        assert lgot == lref
        assert torch.equal(got.buf.series, ref.buf.series)
        for a, b in zip(got.fields(), ref.fields()):              # E, H on the cells (not the padding)
            assert torch.equal(a, b)
        nb, stride, scale_off = store_layout(ref)
        payload = int(ref.info.values_per_slice) * nb
        for j in range(int(ref.info.slices)):                  # slice payloads (not the padding)
            assert torch.equal(got.buf.store[j * stride: j * stride + payload],
                               ref.buf.store[j * stride: j * stride + payload]), (p.name, j)
        sb = int(ref.info.scale_bytes)
        assert torch.equal(got.buf.store[scale_off: scale_off + sb], ref.buf.store[scale_off: scale_off + sb])
        # its record feeds the backward pass, which needs nothing left in the forward's workspace
        gg = got.backward().cpu().numpy()
        gr = ref.backward().cpu().numpy()
        assert np.array_equal(gg, gr)


def test_noalloc_refuses_problems_beyond_its_array():
    require_gpu()
    prob = w.c4(steps=8)
    g = pk.Gradient(prob, "fp32", 1, with_backward=False)
    need = int(g.info.workspace_bytes) - int(g.info.fields_bytes)
    assert need > pk._lib.NOALLOC_SCRATCH_BYTES
    eps = torch.from_numpy(prob.eps).cuda()
    with pytest.raises(pk.FdtdError) as e:
        g.forward_noalloc(eps)
    assert e.value.code == pk._lib.FDTD_EINVAL
