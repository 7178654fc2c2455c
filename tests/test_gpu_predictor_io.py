"""The predictor's native training and file entry points through the C ABI:
bern_pred_train fits the MLP with the library's kernels (the loss falls and
the classes of a separable problem are learned), writes the file that
bern_pred_load reads back (same parameters), and refuses bad inputs."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_14438_amd import bernnn as B  # noqa: E402
from paper_2211_14438_amd import predictor as PR  # noqa: E402


def _records(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8)).astype(np.float32) * 2.0 + 1.0
    y = ((X[:, 0] > 1.0).astype(np.int8) + 2 * (X[:, 3] > 1.0).astype(np.int8)).astype(np.int8)
    return X, y


def test_train_writes_a_file_that_loads(tmp_path):
    X, y = _records(20000, 1)
    path = str(tmp_path / "p.bin")
    pred, losses = B.pred_train(X, y, path=path, epochs=30, batch=2048, lr=1e-2, seed=3, meta='{"test": 1}')
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.3 * losses[0]
    P = PR.read_params(path)
    assert P.shape == (B.N_PARAMS,) and np.all(np.isfinite(P))
    # the normalisation the trainer fixed: the records' mean and std (+1e-3)
    assert np.allclose(P[:8], X.mean(0), atol=1e-4) and np.allclose(P[8:16], X.std(0) + 1e-3, rtol=1e-4)
    cls, _ = B.mlp_classify(torch.tensor(P, device="cuda"), torch.tensor(X, device="cuda"), bf16=False)
    assert (cls.cpu().numpy() == y).mean() > 0.95
    # the file loads into a predictor the pipeline can use; the same seed trains the same bits
    B.Predictor.load(path).close()
    _, again = B.pred_train(X, y, path=str(tmp_path / "q.bin"), epochs=30, batch=2048, lr=1e-2, seed=3,
                            want_predictor=False)
    assert np.array_equal(losses, again)
    assert np.array_equal(PR.read_params(str(tmp_path / "q.bin")), P)
    pred.close()


def test_bad_inputs_refused(tmp_path):
    X, y = _records(100, 2)
    bad = y.copy()
    bad[5] = 4
    with pytest.raises(B.BernError) as ei:
        B.pred_train(X, bad, epochs=1)
    assert ei.value.status == -1
    Xn = X.copy()
    Xn[3, 2] = np.nan
    with pytest.raises(B.BernError) as ei:
        B.pred_train(Xn, y, epochs=1)
    assert ei.value.status == -9
    p = tmp_path / "junk.bin"
    p.write_bytes(b"NOTAPRED" + bytes(64))
    with pytest.raises(B.BernError):
        B.Predictor.load(str(p))
    with pytest.raises(B.BernError):
        B.Predictor.load(str(tmp_path / "missing.bin"))
    # truncated
    X2, y2 = _records(3000, 4)
    B.pred_train(X2, y2, path=str(tmp_path / "t.bin"), epochs=1, batch=1024, want_predictor=False)
    raw = (tmp_path / "t.bin").read_bytes()
    (tmp_path / "t2.bin").write_bytes(raw[: len(raw) // 2])
    with pytest.raises(B.BernError):
        B.Predictor.load(str(tmp_path / "t2.bin"))
    assert os.path.getsize(tmp_path / "t.bin") == 16 + 4 * B.N_PARAMS + 4
