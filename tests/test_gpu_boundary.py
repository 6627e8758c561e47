"""The Python binding rejects arguments the C ABI could not check (device
pointers): host tensors, wrong dtypes and shapes, and batched-decode shot
codes or rows outside the models' arrays raise before anything is launched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2607_27644_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import rbp as mod
    return mod


def test_decode_rejects_host_and_misshapen_tensors(rbp):
    dem = W.workload("cc160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, 8, seed=1)
    with pytest.raises(ValueError, match="GPU"):
        code.decode(dem.priors, syn.cpu(), params)
    with pytest.raises(TypeError):
        code.decode(dem.priors, syn.to(torch.int64), params)
    with pytest.raises(ValueError, match="shape"):
        code.decode(dem.priors, syn[:, :1].contiguous(), params)
    with pytest.raises(ValueError, match="contiguous"):
        code.decode(dem.priors, torch.zeros((2, 8), dtype=torch.int32, device="cuda")[:, ::4], params)
    with pytest.raises(ValueError, match="shape"):
        code.decode(dem.priors[:-1], syn, params)
    with pytest.raises(ValueError, match="GPU"):
        code.decode(dem.priors, syn, params, delta=torch.zeros((8, dem.N)))
    corr, obsp, st = code.decode(dem.priors, syn, params)
    with pytest.raises(ValueError, match="shape"):
        code.decode(dem.priors, syn, params, out=(corr[:4], obsp, st))
    with pytest.raises(ValueError, match="GPU"):
        code.decode(dem.priors, syn, params, out=(corr, obsp, st.cpu()))
    # the outputs of the valid call are untouched by the rejected ones
    corr2, _, _ = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    assert torch.equal(corr, corr2)


def test_decode_multi_rejects_bad_codes_and_rows(rbp):
    dems = [W.workload("cc160"), W.workload("tiny60")]
    codes = [rbp.Code.from_dem(d) for d in dems]
    params = rbp.RelayParams()
    syns = [c.sample(d.priors, 10, seed=i)[0] for i, (c, d) in enumerate(zip(codes, dems))]
    corrs = [torch.zeros((10, rbp.words(d.N)), dtype=torch.int32, device="cuda") for d in dems]
    obsps = [torch.zeros((10, max(rbp.words(d.k), 1)), dtype=torch.int32, device="cuda") for d in dems]
    code_ok = torch.tensor([0, 1] * 10, dtype=torch.uint8, device="cuda")
    idx_ok = torch.arange(20, dtype=torch.int32, device="cuda") // 2
    rbp.decode_multi(codes, [d.priors for d in dems], code_ok, idx_ok, syns, params, corrs, obsps)
    torch.cuda.synchronize()
    bad_code = code_ok.clone()
    bad_code[3] = 2
    with pytest.raises(ValueError, match="shot_code"):
        rbp.decode_multi(codes, [d.priors for d in dems], bad_code, idx_ok, syns, params, corrs, obsps)
    bad_idx = idx_ok.clone()
    bad_idx[5] = 10
    with pytest.raises(ValueError, match="shot_index"):
        rbp.decode_multi(codes, [d.priors for d in dems], code_ok, bad_idx, syns, params, corrs, obsps)
    bad_idx[5] = -1
    with pytest.raises(ValueError, match="shot_index"):
        rbp.decode_multi(codes, [d.priors for d in dems], code_ok, bad_idx, syns, params, corrs, obsps)
    with pytest.raises(ValueError, match="GPU"):
        rbp.decode_multi(codes, [d.priors for d in dems], code_ok.cpu(), idx_ok, syns, params, corrs, obsps)


def test_network_rejects_host_tensors(rbp):
    net = rbp.MLP(64, 32, 160, seed=1)
    x = torch.zeros((4, 2), dtype=torch.int32)
    with pytest.raises(ValueError, match="GPU"):
        net.forward(x)
    with pytest.raises(ValueError, match="shape"):
        net.forward(torch.zeros((4, 3), dtype=torch.int32, device="cuda"))
