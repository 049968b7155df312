"""The entry point that allocates nothing, paid_mlp_loss_grad_noalloc,
against paid_mlp_loss_grad through the C ABI: two calls in a row, the second
with fewer samples, each bit-identical to the allocating entry point (the
same kernels on the same inputs); sizes beyond the fixed working memory and
host arrays are refused before anything is launched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_loss_grad_matches_the_allocating_entry_point():
    import torch

    import paid_1610_09991_amd as P
    dev = torch.device("cuda:0")
    npar = P.mlp_nparams()
    rng = np.random.default_rng(21)
    w = torch.tensor(rng.normal(0.0, 0.1, npar).astype(np.float32), device=dev)
    sizes = (P.NOALLOC_MAX_N, 300)  # the largest input, then a smaller one
    data = [(torch.tensor(rng.normal(size=(n, 7)).astype(np.float32), device=dev),
             torch.tensor(rng.normal(size=(n, 256)).astype(np.float32), device=dev)) for n in sizes]
    with P.Context() as c:
        refs = []
        for x, y in data:
            g = torch.zeros(npar, dtype=torch.float32, device=dev)
            loss, _ = c.mlp_loss_grad(w, x, y, g)
            refs.append((loss, g))
        got = []
        for x, y in data:  # two calls in a row on the same fixed array
            g = torch.full((npar,), float("nan"), dtype=torch.float32, device=dev)
            got.append((c.mlp_loss_grad_noalloc(w, x, y, g), g))
        torch.cuda.synchronize()
        for (lr, gr), (ln, gn), n in zip(refs, got, sizes):
            assert ln == lr, (n, ln, lr)
            assert torch.equal(gn, gr), n
            assert torch.isfinite(gn).all()
        # refused: more samples than the fixed array holds, host arrays
        n = P.NOALLOC_MAX_N + 1
        x = torch.zeros((n, 7), dtype=torch.float32, device=dev)
        y = torch.zeros((n, 256), dtype=torch.float32, device=dev)
        g = torch.zeros(npar, dtype=torch.float32, device=dev)
        with pytest.raises(P.PaidError) as ei:
            c.mlp_loss_grad_noalloc(w, x, y, g)
        assert ei.value.code == P.EINVAL
        xh, yh = data[1][0].cpu().numpy(), data[1][1].cpu().numpy()
        with pytest.raises(P.PaidError) as ei:
            c.mlp_loss_grad_noalloc(w, xh, yh, g)
        assert ei.value.code == P.EINVAL
