"""The allocation-free network evaluation (ewbem_mlp_eval_noalloc) against
ewbem_mlp_eval through the C-ABI: the same kernels on buffers carved from
the library's static scratch instead of allocated ones, so outputs, loss
and gradient must agree bit for bit.  Two calls in a row, the second on a
smaller batch and a narrower network (the scratch keeps the first call's
contents), then a request larger than the scratch, which must be refused
before any work is enqueued."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _net(dims, rng):
    p = []
    for l in range(len(dims) - 1):
        p.append(rng.standard_normal(dims[l + 1] * dims[l]) / np.sqrt(dims[l]))
        p.append(rng.standard_normal(dims[l + 1]) * 0.1)
    return np.concatenate(p).astype(np.float32)


def _both(c, torch, dev, dims, batch, seed):
    rng = np.random.default_rng(seed)
    p = torch.from_numpy(_net(dims, rng)).to(dev)
    x = torch.from_numpy(rng.standard_normal(batch * dims[0]).astype(np.float32)).to(dev)
    t = torch.from_numpy(rng.standard_normal(batch * dims[-1]).astype(np.float32)).to(dev)
    out = {}
    for name, na in (("alloc", False), ("noalloc", True)):
        y = torch.full((batch * dims[-1],), float("nan"), dtype=torch.float32, device=dev)
        g = torch.full((p.numel(),), float("nan"), dtype=torch.float32, device=dev)
        y2 = torch.full_like(y, float("nan"))
        loss = c.mlp_eval(dims, p, x, y, target=t, grad=g, noalloc=na)
        c.mlp_eval(dims, p, x, y2, noalloc=na)  # forward only
        out[name] = (y.cpu().numpy(), g.cpu().numpy(), loss, y2.cpu().numpy())
    return out


def test_noalloc_matches_allocating_eval():
    import torch
    from paper_1212_3032_amd import ewbem as E
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    c = E.Context(0)
    for dims, batch, seed in (([386, 256, 256, 256, 128], 3000, 1), ([33, 70, 17], 130, 2)):
        print(f"mlp_eval_noalloc dims={dims} batch={batch}", flush=True)
        sys.stdout.flush()
        o = _both(c, torch, dev, dims, batch, seed)
        ya, ga, la, fa = o["alloc"]
        yn, gn, ln, fn = o["noalloc"]
        assert np.isfinite(ya).all() and np.isfinite(ga).all()
        assert np.array_equal(ya, yn) and np.array_equal(ga, gn) and la == ln
        assert np.array_equal(fa, fn) and np.array_equal(fa, ya)
    # beyond the scratch: 2 x 60,000 x 768 hidden floats alone exceed 32 MiB
    dims = [386, 256, 256, 256, 128]
    batch = 60000
    p = torch.zeros(sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(4)), dtype=torch.float32, device=dev)
    x = torch.zeros(batch * dims[0], dtype=torch.float32, device=dev)
    y = torch.zeros(batch * dims[-1], dtype=torch.float32, device=dev)
    with pytest.raises(E.EwbemError) as e:
        c.mlp_eval(dims, p, x, y, noalloc=True)
    assert e.value.status == E.EINVAL and "scratch" in str(e.value)
    # an empty batch zeroes the gradient
    g = torch.full((p.numel(),), 7.0, dtype=torch.float32, device=dev)
    assert c.mlp_eval(dims, p, x[:0], y[:0], target=y[:0], grad=g, noalloc=True) == 0.0
    assert float(g.abs().max()) == 0.0
    c.close()
