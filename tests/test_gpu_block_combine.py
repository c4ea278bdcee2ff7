"""bem_block_combine, the column-scaled block sum that forms the inverse iterations' right-hand
sides on the device, against numpy: 1, 3, 11 and 64 blocks with per-column complex factors, a
single row, a ragged column count, a row stride larger than m, the output written over the
first block; and its argument errors (no blocks, more than 64, mismatched strides, an output
overlapping a block at another stride)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _blocks(rng, nb, n, ld):
    return [rng.standard_normal((n, ld)) + 1j * rng.standard_normal((n, ld)) for _ in range(nb)]


@pytest.mark.parametrize("nb,n,m,ld", [(1, 1, 3, 3), (3, 1000, 33, 40), (11, 4097, 32, 32), (64, 300, 7, 9)])
def test_block_combine_matches_numpy(nb, n, m, ld):
    import torch

    from paper_1906_03938_amd import _lib

    rng = np.random.default_rng(nb * 1000 + m)
    X = _blocks(rng, nb, n, ld)
    C = rng.standard_normal((nb, m)) + 1j * rng.standard_normal((nb, m))
    Xd = [torch.from_numpy(x).to("cuda")[:, :m] for x in X]
    out = _lib.block_combine(Xd, C).cpu().numpy()
    ref = sum(C[b][None, :] * X[b][:, :m] for b in range(nb))
    scale = sum(np.abs(C[b])[None, :] * np.abs(X[b][:, :m]) for b in range(nb))
    err = np.max(np.abs(out - ref) / scale)
    print(f"nb={nb} n={n} m={m} ld={ld} max error / sum of |terms| {err:.2e}", flush=True)
    assert err <= 4 * nb * 2.0 ** -52
    # the output over the first block (same row stride)
    first = Xd[0]
    _lib.block_combine(Xd, C, out=first)
    assert np.array_equal(first.cpu().numpy(), out)


def test_block_combine_errors():
    import torch

    import paper_1906_03938_amd as bem
    from paper_1906_03938_amd import _lib

    a = torch.zeros((4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        _lib.block_combine([], np.zeros((0, 3)))
    with pytest.raises(bem.BemError, match="EINVAL"):
        _lib.block_combine([a] * 65, np.ones((65, 3)))
    wide = torch.zeros((4, 5), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        _lib.block_combine([a, wide[:, :3]], np.ones((2, 3)))
    # an output overlapping a block at another row stride
    with pytest.raises(bem.BemError, match="EINVAL"):
        _lib.block_combine([wide[:, :3]], np.ones((1, 3)), out=wide.view(-1)[:12].view(4, 3))
