"""The allocation-free forward pass of the warm-start network
(mlp_forward_noalloc, through the C-ABI) against the allocating one
(mlp_forward): two calls in a row, the second with fewer rows, each equal
to the allocating pass on the same rows (same kernels, same inputs:
bitwise); rows beyond the scratch array's limit are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_forward_on_two_calls():
    import torch

    from paper_2410_13055_amd import gridplan

    torch.cuda.set_device(0)
    st = gridplan.current_stream()
    net = gridplan.MLP(843, 512, 3, 336, seed=3, stream=st)
    try:
        rng = np.random.default_rng(5)
        # a standardisation that is not the identity, so the input cast and
        # the output unscale both act
        net.set_scaling(rng.normal(0, 1, 843).astype(np.float32), rng.uniform(0.5, 2, 843).astype(np.float32),
                        rng.normal(0, 1, 336).astype(np.float32), rng.uniform(0.5, 2, 336).astype(np.float32))
        cap = net.noalloc_rows()
        print(f"\n[gpu] allocation-free forward: at most {cap} rows", flush=True)
        assert cap > 4000
        for rows in (4000, 1037):
            X = torch.from_numpy(rng.normal(0, 1, (rows, 843)).astype(np.float32)).cuda()
            Y_ref = net.forward(X)
            Y = torch.full((rows, 336), float("nan"), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            got = net.forward_noalloc(X, Y)
            torch.cuda.synchronize()
            assert got == cap
            assert torch.isfinite(Y).all()
            assert torch.equal(Y, Y_ref), float((Y - Y_ref).abs().max())
        X = torch.zeros((cap + 1, 843), dtype=torch.float32, device="cuda")
        Y = torch.zeros((cap + 1, 336), dtype=torch.float32, device="cuda")
        with pytest.raises(gridplan.GridplanError) as ei:
            net.forward_noalloc(X, Y)
        assert ei.value.code == gridplan.GP_EINVAL and "scratch" in str(ei.value)
    finally:
        net.close()
