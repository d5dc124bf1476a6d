"""The no-allocation training step (pcsir_mlp_train_step_static) against the
workspace one (pcsir_mlp_train_step): the same kernels on the same inputs, so
parameters, Adam moments, gradients and loss must agree bit for bit, on two
calls in a row, the second with a smaller batch than the first (the device
array then still holds the first call's larger contents). A batch above the
array's maximum is rejected before any work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_5541_amd import lib
    lib()


def _rows(rng, n):
    import torch
    X = torch.from_numpy(rng.normal(0.0, 0.5, size=(n, 256)).astype(np.float32)).to(torch.bfloat16).cuda()
    y = torch.from_numpy(rng.normal(0.0, 0.3, size=n).astype(np.float32)).cuda()
    return X.contiguous(), y


def _same(a, b, what):
    import torch
    assert torch.equal(a, b), f"{what}: max |d| = {(a - b).abs().max().item()}"


def test_static_train_step_matches_workspace_step():
    import torch

    from paper_1310_5541_amd import MLPTrainer, mlp_param_count
    rng = np.random.default_rng(20240)
    p0 = torch.from_numpy(rng.normal(0.0, 0.06, size=mlp_param_count()).astype(np.float32)).cuda()
    X1, y1 = _rows(rng, 1024)
    X2, y2 = _rows(rng, 192)
    lr = 1e-3
    print("case no_alloc: batch 1024 then 192", flush=True)
    ref = MLPTrainer(p0, batch=1024)
    st = MLPTrainer(p0, batch=1024)
    ref.step(X1, y1, lr)
    assert st.step_static(X1, y1, lr) == 0
    torch.cuda.synchronize()
    for name in ("params", "m", "v", "grad", "loss"):
        _same(getattr(st, name), getattr(ref, name), f"call 1 {name}")
    # second call, smaller batch: the workspace path continues in a trainer of that batch
    ref2 = MLPTrainer(ref.params, batch=192)
    ref2.m.copy_(ref.m)
    ref2.v.copy_(ref.v)
    ref2.t = ref.t
    ref2.step(X2, y2, lr)
    assert st.step_static(X2, y2, lr) == 0
    torch.cuda.synchronize()
    for name in ("params", "m", "v", "grad", "loss"):
        _same(getattr(st, name), getattr(ref2, name), f"call 2 {name}")
    assert not torch.equal(st.params, ref.params)  # the second step moved the parameters


def test_static_train_step_rejects_large_and_ragged_batches():
    import torch

    from paper_1310_5541_amd import MLPTrainer, mlp_param_count
    rng = np.random.default_rng(7)
    p0 = torch.from_numpy(rng.normal(0.0, 0.06, size=mlp_param_count()).astype(np.float32)).cuda()
    tr = MLPTrainer(p0, batch=64)
    before = tr.params.clone()
    X, y = _rows(rng, 1088)
    assert tr.step_static(X, y, 1e-3) == -2  # PCSIR_E_NOMEM: above the array's 1024 rows
    Xr, yr = _rows(rng, 100)
    assert tr.step_static(Xr, yr, 1e-3) == -1  # PCSIR_E_INVAL: not a multiple of 64
    torch.cuda.synchronize()
    _same(tr.params, before, "parameters after rejected calls")
