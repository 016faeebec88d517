"""GPU check of ffs_evaluate_noalloc, the decode entry point that allocates
nothing, against ffs_evaluate on the same rows: two calls in a row, the
second with a smaller input (another instance, fewer rows), then rows that
are not permutations, then an instance beyond its state limit."""
import numpy as np
import pytest

from gpu_util import ensure_built, make_ctx, say
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu

ISL = [inputs.cellular(3, 3, 0.9, 0.1), inputs.pseudo(2, 0.75, 0.0)]


def _reference(m, p, perms):
    ctx = make_ctx([dict(m=m, p=p, islands=ISL, interval=0)])
    out, rc = ctx.evaluate(0, perms, check=False)
    out = out.cpu().numpy()
    ctx.close()
    return out, rc


def test_noalloc_decode_matches_evaluate():
    import torch

    from paper_1903_10722_amd.binding import FFS_EINVAL, FFS_EUNSUPPORTED, FFS_OK, FFSError, evaluate_noalloc
    ensure_built()
    dev = torch.device("cuda", 0)
    # first call: the large shape, enough rows for the lane mapping; second
    # call: a smaller instance and fewer rows (per-stage mapping)
    for n, S, lo, hi, rows, seed in ((500, 10, 3, 5, 70000, 1), (100, 5, 1, 5, 3001, 2)):
        m, p = inputs.make_instance(n, S, lo, hi, seed=seed)
        perms = inputs.random_perms(rows, n, seed=seed + 10)
        say(f"[noalloc] n={n} S={S} rows={rows}")
        t = torch.from_numpy(perms).to(dev)
        out = torch.full((rows,), -7, dtype=torch.int32, device=dev)
        rc = evaluate_noalloc(m, p, t, out)
        torch.cuda.synchronize()
        want, rc_ref = _reference(m, p, perms)
        assert rc == FFS_OK and rc_ref == FFS_OK
        assert np.array_equal(out.cpu().numpy(), want)
    # rows that are not permutations: -1 on those rows, FFS_EINVAL, like ffs_evaluate
    m, p = inputs.make_instance(30, 4, 1, 4, seed=5)
    perms = inputs.random_perms(200, 30, seed=3)
    perms[7, 4] = 30
    perms[51, 3] = perms[51, 9]
    say("[noalloc] invalid rows")
    out = torch.zeros(200, dtype=torch.int32, device=dev)
    rc = evaluate_noalloc(m, p, torch.from_numpy(perms).to(dev), out)
    want, rc_ref = _reference(m, p, perms)
    assert rc == FFS_EINVAL and rc_ref == FFS_EINVAL
    assert np.array_equal(out.cpu().numpy(), want) and (want[[7, 51]] == -1).all()
    # beyond the 1 MiB of state: refused before any device work
    m, p = inputs.make_instance(4096, 64, 1, 2, p_hi=3, seed=1)
    with pytest.raises(FFSError) as e:
        evaluate_noalloc(m, p, torch.zeros((1, 4096), dtype=torch.int32, device=dev),
                         torch.zeros(1, dtype=torch.int32, device=dev))
    assert e.value.code == FFS_EUNSUPPORTED
