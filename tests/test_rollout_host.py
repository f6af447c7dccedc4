"""Host-side logic of the differentiable rollout that needs no GPU: the
checkpoint slots carved from one allocation, and the argument checks of the
binding."""
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


def _fake_grid(has_body=True):
    """A binding-level Grid with the layouts of a 2D 8 x 6 grid whose x axis
    is bounded, on the CPU and with no library handle: every call below must
    be refused by the argument checks before anything reaches the library."""
    from paper_2505_23940_amd import Grid
    g = Grid.__new__(Grid)
    g.device = torch.device("cpu")
    g.dim = 2
    g.dtype = torch.float32
    g.layouts = [((1, 6, 9), (54, 9, 1), 0), ((1, 6, 8), (48, 8, 1), 0)]
    g.pshape = (1, 6, 8)
    g.has_body = has_body
    g.h = None
    g._info = torch.zeros(8, dtype=torch.float64)
    return g


def _good(g):
    u = [torch.zeros(l[0], dtype=torch.float32) for l in g.layouts]
    p = torch.zeros(g.pshape, dtype=torch.float64)
    body = torch.zeros(6, dtype=torch.float64)
    kc = torch.zeros(6, dtype=torch.float64)
    return u, p, body, kc


@pytest.mark.parametrize("bad", ["p_dtype", "p_shape", "p_out_shape", "u_out_dtype", "body_short",
                                 "body_missing", "kc_float32", "info_short", "p_noncontig"])
def test_step_rejects_malformed_tensors_before_launch(bad):
    g = _fake_grid()
    u, p, body, kc = _good(g)
    kw = {}
    if bad == "p_dtype":
        p = p.float()
    elif bad == "p_shape":
        p = torch.zeros((1, 6, 9), dtype=torch.float64)
    elif bad == "p_out_shape":
        kw["p_out"] = torch.zeros(10, dtype=torch.float64)
    elif bad == "u_out_dtype":
        kw["u_out"] = [x.double() for x in u]
    elif bad == "body_short":
        body = torch.zeros(3, dtype=torch.float64)
    elif bad == "body_missing":
        body = None
    elif bad == "kc_float32":
        kc = kc.float()
    elif bad == "info_short":
        kw["info"] = torch.zeros(4, dtype=torch.float64)
    elif bad == "p_noncontig":
        p = torch.zeros((1, 8, 6), dtype=torch.float64).transpose(1, 2)
    with pytest.raises(ValueError):
        g.step(u, p, None, body, kc, **kw)


@pytest.mark.parametrize("bad", ["ubar_out_shape", "ubar_in_dtype", "fbbar_len", "bodybar_in_missing",
                                 "kcbar_short", "dF_short", "mu_shape"])
def test_step_adjoint_rejects_malformed_tensors_before_launch(bad):
    g = _fake_grid()
    u, p, body, kc = _good(g)
    ubo = [x.clone() for x in u]
    ubi = [x.clone() for x in u]
    bbo, bbi, kcb = body.clone(), body.clone(), kc.clone()
    dF = torch.zeros(3, dtype=torch.float64)
    kw = {"fbbar": [x.clone() for x in u], "kcbar": kcb, "mu": p.clone()}
    if bad == "ubar_out_shape":
        ubo[1] = torch.zeros((1, 6, 9), dtype=torch.float32)
    elif bad == "ubar_in_dtype":
        ubi = [x.double() for x in ubi]
    elif bad == "fbbar_len":
        kw["fbbar"] = kw["fbbar"][:1]
    elif bad == "bodybar_in_missing":
        bbi = None
    elif bad == "kcbar_short":
        kw["kcbar"] = torch.zeros(2, dtype=torch.float64)
    elif bad == "dF_short":
        dF = torch.zeros(1, dtype=torch.float64)
    elif bad == "mu_shape":
        kw["mu"] = torch.zeros(48, dtype=torch.float64)
    with pytest.raises(ValueError):
        g.step_adjoint(u, None, body, kc, ubo, bbo, dF, ubi, bbi, **kw)
