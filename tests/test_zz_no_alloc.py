"""The no-allocation soft forward (aerl_soft_forward_noalloc): called through
the C ABI, it must give what aerl_soft_forward gives on the same inputs, bit
for bit (same kernels, same reduction order), and stay within the soft-path
tolerance of the fp64 oracle; two calls in a row, the second smaller, show
that the shared scratch array carries nothing from one call to the next.
Sizes past the array's limit are refused before any launch."""
import numpy as np
import pytest

import oracle
from paper_2406_01821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2406_01821_amd.aerl import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _params(pop, dev):
    import torch
    return [torch.tensor(a, device=dev) for a in (pop.coef, pop.coef2, pop.theta)]


def _both(ctx, w):
    import torch
    ds = ctx.upload_dataset(w.data)
    p = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    c1, c2, th = _params(w.pop, ctx.device)
    ref = ctx.soft_forward(ds, p, c1, c2, th)
    out = torch.full((w.pop.n_sets,), float("nan"), dtype=torch.float32, device=ctx.device)
    ctx.soft_forward_noalloc(ds, p, c1, c2, th, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_matches_the_workspace_entry_twice(ctx):
    big = synth.soft_workload(11, n=20_000, nf=12, n_sets=96, n_rules=6, n_conds=3)
    small = synth.tiny(12, n=700, nf=5, n_classes=3, n_sets=9, rules=(1, 5), conds=(1, 3),
                       ff_frac=0.4)
    for w in (big, small):
        print(f"no-alloc soft forward: {w.name}, {w.pop.n_sets} sets", flush=True)
        ref, got = _both(ctx, w)
        assert np.array_equal(ref, got)
        tau = oracle.tau(w.data.x)
        l64 = oracle.soft_forward(w.data.x, w.data.y, tau, w.data.n_classes, w.pop)
        assert np.all(np.abs(got - l64) <= 1e-5 * np.abs(l64) + 1e-6)


def test_noalloc_refuses_what_does_not_fit(ctx):
    import torch
    from paper_2406_01821_amd.aerl import AerlError, AERL_ENOMEM, AERL_NOALLOC_SCRATCH_BYTES
    # 600,000 one-condition rule sets: 9.6 MB of condition records plus at
    # least one group of fp64 partials per class region (2 x 600,000 x 8 B),
    # past the 16 MiB scratch array
    w = synth.soft_workload(13, n=1 << 15, nf=8, n_sets=600_000, n_rules=1, n_conds=1)
    ds = ctx.upload_dataset(w.data)
    p = ctx.pack_population(w.pop, 8, 2)
    assert ctx.soft_workspace(ds, p, False).numel() > AERL_NOALLOC_SCRATCH_BYTES
    c1, c2, th = _params(w.pop, ctx.device)
    out = torch.zeros(w.pop.n_sets, dtype=torch.float32, device=ctx.device)
    with pytest.raises(AerlError) as e:
        ctx.soft_forward_noalloc(ds, p, c1, c2, th, out)
    assert e.value.status == AERL_ENOMEM
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
