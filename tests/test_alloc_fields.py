"""The binding's pooled field allocation (alloc_fields), on the host: every
view has the requested shape and dtype, is contiguous, starts on the
requested boundary, and owns its own bytes."""
import pytest
import torch

from paper_2010_01545_amd import pwadvect as pw


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("count,shape,align", [(1, (3, 4, 5), 256), (6, (9, 7, 11), 4096), (12, (5, 6, 68), 512),
                                               (3, (0, 4, 4), 256)])
def test_views_are_aligned_contiguous_and_disjoint(count, shape, align, dtype):
    ts = pw.alloc_fields(count, shape, dtype, device="cpu", align=align)
    assert len(ts) == count
    esize = ts[0].element_size()
    nbytes = ts[0].numel() * esize
    spans = []
    for t in ts:
        assert tuple(t.shape) == shape and t.dtype == dtype and t.is_contiguous()
        assert t.data_ptr() % align == 0
        spans.append((t.data_ptr(), t.data_ptr() + nbytes))
    spans.sort()
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0
    if nbytes:
        for q, t in enumerate(ts):
            t.fill_(q + 1)
        for q, t in enumerate(ts):
            assert torch.all(t == q + 1)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        pw.alloc_fields(0, (2, 2, 2), torch.float64, device="cpu")
    with pytest.raises(ValueError):
        pw.alloc_fields(2, (2, 2, 2), torch.float64, device="cpu", align=100)
    with pytest.raises(ValueError):
        pw.alloc_fields(2, (2, -1, 2), torch.float64, device="cpu")
