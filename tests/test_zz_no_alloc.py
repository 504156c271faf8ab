"""The allocation-free surrogate prediction (sur_predict_noalloc) against sur_predict.

Both run the same kernels on the same data (the forward pass of the
5000 -> 256 -> 256 -> 1 network with the same split of the long sums); the
allocation-free one takes its workspaces from the library's fixed scratch
array.  Two calls in a row, the second with a smaller batch (the array keeps
the first call's contents), must each give exactly sur_predict's result; a
batch whose workspaces exceed the array is refused with CTM_EINVAL.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctm_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_14414_amd as m
    return m


def test_noalloc_prediction_equals_prediction(ctm_mod):
    rng = np.random.default_rng(11)
    net = ctm_mod.Surrogate(5000, 256, seed=3)
    # a few training steps so that the target statistics are not the identity
    Xt = torch.tensor(rng.standard_normal((32, 5000)), dtype=torch.float32)
    tt = torch.tensor(rng.standard_normal(32) * 0.1 - 0.4, dtype=torch.float32)
    net.train(Xt, tt, 5)
    for batch in (64, 8):
        X = torch.tensor(rng.standard_normal((batch, 5000)), dtype=torch.float32)
        y_ref = net.predict(X)
        y = net.predict_noalloc(X)
        print(f"batch {batch}: max |y - y_ref| = {(y - y_ref).abs().max().item():.3e}")
        assert y.shape == y_ref.shape and torch.equal(y, y_ref)
    with pytest.raises(ctm_mod.CTMError) as err:
        net.predict_noalloc(torch.zeros((4096, 5000), dtype=torch.float32))
    assert err.value.code == -1 and "maximum" in str(err.value)
    # still usable after the refusal
    X = torch.tensor(rng.standard_normal((3, 5000)), dtype=torch.float32)
    assert torch.equal(net.predict_noalloc(X), net.predict(X))
    net.close()
