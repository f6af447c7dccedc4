"""Host-side logic of the differentiable rollout that needs no GPU: the
checkpoint slots carved from one allocation."""
import pytest
import torch

from paper_2505_23940_amd.rollout import _slots_like


@pytest.mark.parametrize("shape,dtype", [((160, 129, 192), torch.float32), ((7, 13, 33), torch.float32),
                                         ((67, 19, 9), torch.float64), ((6,), torch.float64)])
def test_checkpoint_slots_are_aligned_disjoint_and_contiguous(shape, dtype):
    x = torch.empty(shape, dtype=dtype)
    slots = _slots_like(x, 4)
    assert len(slots) == 4
    base = slots[0].data_ptr()
    nbytes = x.numel() * x.element_size()
    for s, t in enumerate(slots):
        assert t.shape == x.shape and t.dtype == x.dtype and t.is_contiguous()
        assert (t.data_ptr() - base) % 256 == 0          # same alignment as an allocation of its own
        t.fill_(float(s + 1))
    # writing one slot leaves the others untouched (no overlap)
    for s, t in enumerate(slots):
        assert float(t.min()) == float(t.max()) == float(s + 1)
    ends = sorted((t.data_ptr(), t.data_ptr() + nbytes) for t in slots)
    assert all(a[1] <= b[0] for a, b in zip(ends, ends[1:]))
