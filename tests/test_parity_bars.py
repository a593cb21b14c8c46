"""The fit clauses of the parity bars (tests/parity.py), on the CPU: the FP64
oracle's own fit, rounded to FP32, passes them; each planted deviation of the
kind a wrong or sloppy fit makes is caught by the clause meant for it."""
import numpy as np
import pytest

from conftest import cached_oracle

DIAG = [0, 2, 5, 9, 14]


@pytest.fixture(scope="module")
def fit():
    o = cached_oracle("pp_sector")
    m = o["trk_nfit"] > 0
    ref = {k: np.asarray(o[k])[m] for k in ("trk_params", "trk_cov", "trk_chi2", "trk_xref")}
    assert len(ref["trk_chi2"]) > 150
    return ref


def _check(ref, par=None, cov=None, chi2=None):
    import parity
    rep = parity.ParityReport()
    f32 = {k: v.astype(np.float32) for k, v in ref.items()}
    parity.compare_fit(rep, f32["trk_params"] if par is None else par,
                       f32["trk_cov"] if cov is None else cov,
                       f32["trk_chi2"] if chi2 is None else chi2, f32["trk_xref"],
                       ref["trk_params"], ref["trk_cov"], ref["trk_chi2"], ref["trk_xref"])
    return rep


def test_fp32_rounding_of_the_oracle_passes(fit):
    rep = _check(fit)
    assert rep.ok, rep.get("failures")
    assert rep["param_within_fraction"] == 1.0


def test_relative_error_on_one_percent_fails(fit):
    par = fit["trk_params"].copy()
    idx = np.arange(0, len(par), 100)
    par[idx, 4] *= 1 + 3e-4  # q/pT off by 3e-4 relative on 1% of the tracklets
    rep = _check(fit, par=par)
    assert not rep.ok and any("within 1e-4" in f for f in rep["failures"])


def test_one_large_shift_fails(fit):
    par = fit["trk_params"].copy()
    sig = np.sqrt(fit["trk_cov"][:, DIAG])
    t = int(np.argmax(np.abs(par[:, 0])))
    par[t, 0] += 0.3 * sig[t, 0]  # y off by 0.3 sigma on one tracklet
    rep = _check(fit, par=par)
    assert not rep.ok and any("0.21 sigma" in f for f in rep["failures"])


def test_moderate_shift_on_a_few_fails(fit):
    par = fit["trk_params"].copy()
    sig = np.sqrt(fit["trk_cov"][:, DIAG])
    idx = np.arange(0, len(par), len(par) // 3)[:3]
    par[idx, 2] += 0.15 * sig[idx, 2]  # sin(phi) off by 0.15 sigma on 3 tracklets
    par[idx, 2] += 2e-4 * np.maximum(np.abs(par[idx, 2]), 1e-2)  # and beyond 1e-4 relative
    rep = _check(fit, par=par)
    assert not rep.ok and any("0.1 sigma" in f for f in rep["failures"])
    assert not any("0.21 sigma" in f for f in rep["failures"])


def test_swapped_tracklets_fail(fit):
    par = fit["trk_params"].copy()
    par[[0, 1]] = par[[1, 0]]
    rep = _check(fit, par=par)
    assert not rep.ok


def test_covariance_and_chi2_clauses(fit):
    cov = fit["trk_cov"].astype(np.float32).copy()
    cov[7, 14] *= 1.06  # q/pT variance off by 6% on one tracklet
    rep = _check(fit, cov=cov)
    assert not rep.ok and any("covariance beyond" in f for f in rep["failures"])
    cov = fit["trk_cov"].astype(np.float32).copy()
    cov[7, 5] *= 1.02  # sin(phi) variance off by 2% on one tracklet: within 4.7e-2, beyond 1e-2
    rep = _check(fit, cov=cov)
    assert not rep.ok and any("within 1e-2" in f for f in rep["failures"])
    chi2 = fit["trk_chi2"].astype(np.float32).copy()
    t = int(np.argmax(chi2))
    chi2[t] *= 1.03
    rep = _check(fit, chi2=chi2)
    assert not rep.ok and any("chi2" in f for f in rep["failures"])
