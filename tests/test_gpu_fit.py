"""GPU: the refit drivers on a small problem.  The adjoint route (batched
forward + path-replay adjoint + Adam) and the LUT route (tables from the walk,
the fused LUT-fit kernel) share the targets; both lower the joint loss of eq.
joint_loss and the spectral error, and report parameter recovery."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_refit_routes_reduce_loss_and_spectral_error():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_27604_amd import fit
    prob = fit.make_problem(n_targets=4, target_paths=1 << 16, seed=11)
    res = fit.run_fit(iters=60, paths=4096, log_every=10, problem=prob)
    hist = res["loss_history"]
    assert hist[-1][1] < 0.9 * hist[0][1], hist
    assert res["spectral_rmse"] < res["spectral_rmse_at_start"], res
    assert set(res["recovery_median_abs_error"]) == {"alpha", "g", "log10_sigma_t", "w"}
    lf = fit.run_lut_fit(iters=60, lut_n=33, lut_paths=1 << 12, problem=prob)
    assert lf["loss_history"][-1][2] < lf["loss_history"][0][2], lf["loss_history"]
    assert lf["spectral_rmse"] < lf["spectral_rmse_at_start"], lf
    assert lf["spectral_rmse_at_start"] == res["spectral_rmse_at_start"]
