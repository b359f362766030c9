"""f2m_gdp_step_noalloc, the GDP iteration for callers that cannot allocate:
through the C ABI its outputs equal f2m_gdp_step's bit for bit, on two calls
in a row (the second on a smaller instance, so it runs over what the first
left in the shared workspace), and sizes above its maximum are refused
before any work is queued."""
import numpy as np
import pytest

from paper_2011_08170_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(ctx, fn_name, xy_d, lam):
    n = xy_d.shape[0]
    out = dict(lam=torch.full((n,), -7, dtype=torch.int64, device="cuda"),
               z4=torch.full((4 * n,), -7, dtype=torch.int64, device="cuda"),
               i4=torch.full((4 * n,), -7, dtype=torch.int32, device="cuda"),
               neg=torch.full((n,), -7, dtype=torch.int32, device="cuda"),
               zero=torch.full((n,), -7, dtype=torch.int32, device="cuda"),
               step=torch.full((n,), -7, dtype=torch.int64, device="cuda"))
    lam_d = torch.from_numpy(lam).cuda()
    fn = getattr(ctx, fn_name)
    rec = fn(xy_d, lam_d, out["lam"], out["z4"], out["i4"], out["neg"], out["zero"], out["step"])
    torch.cuda.synchronize()
    return rec, {k: v.cpu().numpy() for k, v in out.items()}


def test_noalloc_step_equals_gdp_step_twice():
    from paper_2011_08170_amd import f2m
    cases = [(I.uniform(30011, 1000000, 4), 1), (I.clustered(5003, 1000000, 2), 2)]
    with f2m.Context(0) as ctx:
        for xy, seed in cases:
            n = len(xy)
            print("noalloc case n=%d" % n, flush=True)
            xy_d = torch.from_numpy(xy).cuda()
            lam = np.random.default_rng(seed).integers(-3000, 3000, n).astype(np.int64)
            want_rec, want = _run(ctx, "gdp_step", xy_d, lam)
            got_rec, got = _run(ctx, "gdp_step_noalloc", xy_d, lam)
            assert got_rec == want_rec
            for k in want:
                assert np.array_equal(got[k], want[k]), k


def test_noalloc_step_null_outputs_and_limits():
    from paper_2011_08170_amd import f2m
    xy = I.uniform(2000, 100000, 9)
    n = len(xy)
    with f2m.Context(0) as ctx:
        xy_d = torch.from_numpy(xy).cuda()
        lam_d = torch.zeros(n, dtype=torch.int64, device="cuda")
        a = torch.empty(n, dtype=torch.int64, device="cuda")
        b = torch.empty(n, dtype=torch.int64, device="cuda")
        ra = ctx.gdp_step(xy_d, lam_d, a)
        rb = ctx.gdp_step_noalloc(xy_d, lam_d, b)
        assert ra == rb and torch.equal(a, b)
        # refused on the host: nothing is launched
        big = f2m.NOALLOC_MAX_N + 1
        with pytest.raises(f2m.F2MError) as e:
            ctx.gdp_step_noalloc(torch.zeros((big, 2), dtype=torch.int32, device="cuda"),
                                 torch.zeros(big, dtype=torch.int64, device="cuda"),
                                 torch.empty(big, dtype=torch.int64, device="cuda"))
        assert e.value.status == -6   # F2M_ERR_CAPACITY
