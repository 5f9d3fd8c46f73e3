"""GPU: the refit driver (batched forward + path-replay adjoint + Adam) lowers
the joint loss of eq. joint_loss and the spectral error on a small problem."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_refit_reduces_loss_and_spectral_error():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_27604_amd import fit
    res = fit.run_fit(n_targets=4, iters=60, paths=4096, target_paths=1 << 16, seed=11,
                      log_every=10)
    hist = res["loss_history"]
    assert hist[-1][1] < 0.9 * hist[0][1], hist
    assert all(b[1] < a[1] for a, b in zip(hist, hist[1:])), hist
    assert res["spectral_rmse"] < res["spectral_rmse_at_start"], res
