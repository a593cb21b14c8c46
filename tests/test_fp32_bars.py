"""Where the outer fit clauses of the parity bars (tests/parity.py) come from,
reproduced on the CPU from committed files alone.

The FP32 tracklet fit cannot follow the FP64 oracle arbitrarily closely: on
ill-conditioned fits (short, low-pT, steep tracklets with chi2 per degree of
freedom far above 1) FP32 rounding alone moves the result by a fair part of a
sigma.  To measure how far, this test builds two copies of the oracle whose
fit (helix transport, Jacobian, covariance transport, Kalman update, seed,
pickup prediction) is evaluated in FP32, operation by operation:

  * fp32_full: the oracle's own steps with every float operation, literal and
    math function in single precision (full 5x5 covariance products);
  * fp32_sym: the same, with the covariance kept as a symmetric lower
    triangle (each update and transport computes the entries j <= i and
    mirrors them), the form the GPU kernel stores.

Both perform the same operations as the FP64 oracle in exact arithmetic and
differ from each other only in rounding order.  Run on every sector of the
50-collision Pb-Pb slice, over the tracklets whose hit sets equal the FP64
oracle's, their deviations from FP64 bound what rounding alone produces.  The
test asserts that every outer clause of the bars admits these FP32 tails and
is at most 1.5 times the larger of them (the bars are not looser than FP32
rounding explains), and that the 1e-4 clause (99.9% of fitted tracklets) is
met by the bulk of both builds.
"""
import re
import subprocess

import numpy as np
import pytest

import oracle
import parity
from conftest import cached_event, cached_oracle
from paper_2106_03636_amd.params import DEFAULT_PARAMS as P

MARGIN = 1.5
DIAG = [0, 2, 5, 9, 14]
FIT_BEGIN = "/* Helix model for the Kalman filter."
FIT_END = "/* driver "


def _fp32_source(symmetric):
    src = open(oracle._SRC).read()
    a, b = src.index(FIT_BEGIN), src.index(FIT_END)
    fit = src[a:b]
    fit = re.sub(r"\bdouble\b", "float", fit)
    for f in ("sqrt", "asin", "fabs", "floor", "nearbyint"):
        fit = re.sub(r"\b%s\(" % f, "%sf(" % f, fit)
    # floating literals in single precision
    fit = re.sub(r"(?<![\w.])((?:\d+\.\d*|\.\d+)(?:[eE][-+]?\d+)?|\d+[eE][-+]?\d+)(?![\w.])", r"\1f", fit)
    if symmetric:
        old_upd = ("  for (int i = 0; i < 5; ++i)\n    for (int j = 0; j < 5; ++j)\n"
                   "      nc[i * 5 + j] = cov[i * 5 + j] - (K[i][0] * cov[0 * 5 + j] + K[i][1] * cov[1 * 5 + j]);\n")
        new_upd = ("  for (int i = 0; i < 5; ++i)\n    for (int j = 0; j <= i; ++j)\n"
                   "      nc[i * 5 + j] = nc[j * 5 + i] =\n"
                   "          cov[i * 5 + j] - (K[i][0] * cov[0 * 5 + j] + K[i][1] * cov[1 * 5 + j]);\n")
        assert fit.count(old_upd) == 1
        fit = fit.replace(old_upd, new_upd)
        old_tr = ("  for (int i = 0; i < 5; ++i)\n    for (int j = 0; j < 5; ++j) {\n      float s = 0;\n"
                  "      for (int l = 0; l < 5; ++l) s += T[i * 5 + l] * F[j * 5 + l];\n      R[i * 5 + j] = s;\n    }\n")
        new_tr = ("  for (int i = 0; i < 5; ++i)\n    for (int j = 0; j <= i; ++j) {\n      float s = 0;\n"
                  "      for (int l = 0; l < 5; ++l) s += T[i * 5 + l] * F[j * 5 + l];\n"
                  "      R[i * 5 + j] = R[j * 5 + i] = s;\n    }\n")
        assert fit.count(old_tr) == 1
        fit = fit.replace(old_tr, new_tr)
    out = src[:a] + fit + src[b:]
    # the driver copies the (now single-precision) fit results element by element
    for arr, n in (("params", 5), ("cov", 15)):
        old = "memcpy(&res->trk_%s[t * %d], o.%s, sizeof(o.%s));" % (arr, n, arr[:3] if arr == "cov" else "p",
                                                                    arr[:3] if arr == "cov" else "p")
        assert out.count(old) == 1, old
        out = out.replace(old, "for (int q_ = 0; q_ < %d; ++q_) res->trk_%s[t * %d + q_] = o.%s[q_];"
                          % (n, arr, n, arr[:3] if arr == "cov" else "p"))
    return out


def _build(tmp_path, symmetric, fma=False):
    """fma: let the compiler contract a * b + c into fused multiply-adds (the
    GPU compiler does), another rounding order of the same operations."""
    name = ("fp32_sym" if symmetric else "fp32_full") + ("_fma" if fma else "")
    c = tmp_path / (name + ".c")
    c.write_text(_fp32_source(symmetric))
    lib = tmp_path / (name + ".so")
    contract = ["-ffp-contract=fast", "-mfma"] if fma else ["-ffp-contract=off"]
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-shared", "-fPIC"]
                          + contract + ["-w", "-o", str(lib), str(c), "-lm"])
    return str(lib)


def _cpu_has_fma():
    try:
        return " fma " in " %s " % " ".join(l for l in open("/proc/cpuinfo") if l.startswith("flags"))
    except OSError:
        return False


def _run_with(lib, ev):
    saved = (oracle._LIB, oracle._lib)
    oracle._LIB, oracle._lib = lib, None
    try:
        return oracle.run_event(ev, P)
    finally:
        oracle._LIB, oracle._lib = saved


def _tails(o64, o32):
    """Deviation statistics of an FP32 build over tracklets with the FP64 hit sets."""
    K = o64["n_tracklets"]
    assert o32["n_tracklets"] == K and np.array_equal(o32["trk_start"], o64["trk_start"])
    same = ~parity.hit_set_diff(parity.oracle_hit_pairs(o32), parity.oracle_hit_pairs(o64), K)
    same &= (o32["trk_nfit"] == o64["trk_nfit"]) & (o64["trk_nfit"] > 0)
    fitted = int((o64["trk_nfit"] > 0).sum())
    gp = o32["trk_params"][same].astype(np.float32).astype(np.float64)
    op = o64["trk_params"][same]
    sig = np.sqrt(np.abs(o64["trk_cov"][same][:, DIAG]))
    dp = np.abs(gp - op)
    tol = parity.PARAM_RTOL * np.maximum(np.abs(op), parity.PARAM_FLOORS)
    beyond_tol = dp > tol
    dps = np.where(beyond_tol, dp / np.maximum(sig, 1e-30), 0.0).max(axis=1)
    gc = o32["trk_cov"][same][:, DIAG].astype(np.float32).astype(np.float64)
    oc = o64["trk_cov"][same][:, DIAG]
    crel = (np.abs(gc - oc) / np.maximum(np.abs(oc), 1e-12)).max(axis=1)
    gx = o32["trk_chi2"][same].astype(np.float32).astype(np.float64)
    xrel = np.abs(gx - o64["trk_chi2"][same]) / np.maximum(np.abs(o64["trk_chi2"][same]), 1.0)
    return dict(n=int(same.sum()), matched=float(same.sum()) / fitted,
                within_1e4=float((~beyond_tol.any(axis=1)).mean()),
                beyond_0p1_sigma=float((dps > parity.PARAM_SIGMA).mean()), max_sigma=float(dps.max()),
                cov_within_1e3=float((crel <= parity.COV_RTOL).mean()),
                cov_within_1e2=float((crel <= parity.COV_RTOL_MID).mean()),
                cov_max=float(crel.max()), chi2_max=float(xrel.max()),
                chi2_within_1e3=float((xrel <= parity.CHI2_RTOL).mean()))


@pytest.fixture(scope="module")
def tails(tmp_path_factory):
    tmp = tmp_path_factory.mktemp("fp32")
    ev = cached_event("pbpb_timeframe_50")
    o64 = oracle.run_event(ev, P)
    out = {}
    for sym in (False, True):
        o32 = _run_with(_build(tmp, sym), ev)
        out["sym" if sym else "full"] = _tails(o64, o32)
        del o32
    print("FP32 tails on %d clusters:" % ev.n, out)
    return out


def test_fp32_builds_match_almost_every_hit_set(tails):
    for t in tails.values():
        assert t["n"] > 500000 and t["matched"] >= parity.MIN_MATCHED_FRACTION


def _worst(tails, key, fn=max):
    return fn(t[key] for t in tails.values())


def test_sigma_clauses_are_no_looser_than_fp32(tails):
    assert parity.PARAM_SIGMA_ALL <= 1.05 * _worst(tails, "max_sigma")
    assert 1.0 - parity.MIN_SIGMA_FRACTION <= 1.5 * _worst(tails, "beyond_0p1_sigma")


def test_covariance_clauses_are_no_looser_than_fp32(tails):
    assert parity.COV_RTOL_ALL <= 1.05 * _worst(tails, "cov_max")
    assert 1.0 - parity.MIN_COV_FRACTION <= 1.1 * (1.0 - _worst(tails, "cov_within_1e3", min))
    assert 1.0 - parity.MIN_COV_MID_FRACTION <= 1.5 * (1.0 - _worst(tails, "cov_within_1e2", min))


def test_chi2_clauses_are_no_looser_than_fp32(tails):
    assert parity.CHI2_RTOL_ALL <= 1.05 * _worst(tails, "chi2_max")
    assert 1.0 - parity.MIN_CHI2_FRACTION <= 1.5 * (1.0 - _worst(tails, "chi2_within_1e3", min))


def test_relative_clause_is_the_stated_tolerance(tails):
    """The 1e-4 relative clause is the tolerance the fit is held to (99.9% of
    fitted tracklets), not derived from FP32 tails: FP32 in absolute
    coordinates reaches only about 90% there, which is why the kernel keeps
    its state relative to exact integer references."""
    assert parity.PARAM_RTOL == 1e-4 and parity.MIN_WITHIN_FRACTION == 0.999
    assert _worst(tails, "within_1e4", min) < 0.95


# ----------------------------------------------------------------------------
# the refit's covariance clauses (parity.REFIT_*)

def _refit_with(lib, ev, o):
    import synth
    saved = (oracle._LIB, oracle._lib)
    if lib:
        oracle._LIB, oracle._lib = lib, None
    try:
        k = float(np.float32(-np.float32(synth.KAPPA) * np.float32(ev.bz)))
        return oracle.refit_tracks(o["track_first_hit"], o["track_n_hits"], o["track_hits"], ev.y, ev.z, ev.row,
                                   ev.row_x.astype(np.float64), k, P)
    finally:
        oracle._LIB, oracle._lib = saved


@pytest.fixture(scope="module")
def refit_tails(tmp_path_factory):
    """Covariance deviations of FP32 builds of the oracle's refit from its
    FP64 refit, over the tracks of the 50-collision frame (the oracle
    tracker's): per build, inner (pass 2) and outer (pass 1) states."""
    tmp = tmp_path_factory.mktemp("fp32_refit")
    ev = cached_event("pbpb_timeframe_50")
    o = cached_oracle("pbpb_timeframe_50")
    r64 = _refit_with(None, ev, o)
    cov0 = np.array([float(np.float32(v)) for v in P["cov0"]])
    out = {}
    for sym in (False, True):
        for fma in ((False, True) if _cpu_has_fma() else (False,)):
            r32 = _refit_with(_build(tmp, sym, fma), ev, o)
            both = r64["ok"].astype(bool) & r32["ok"].astype(bool)
            for end, key in (("inner", "cov"), ("outer", "cov_out")):
                oc = r64[key][both][:, DIAG]
                gc = r32[key][both][:, DIAG].astype(np.float32).astype(np.float64)
                crel_el = np.abs(gc - oc) / np.abs(oc)
                crel = crel_el.max(axis=1)
                big = crel_el > parity.COV_RTOL_MID
                cond = parity.FP32_EPS * cov0[None, :] / np.abs(oc)
                out[(sym, fma, end)] = dict(
                    n=int(both.sum()), within_1e3=float((crel <= parity.COV_RTOL).mean()),
                    within_1e2=float((crel <= parity.COV_RTOL_MID).mean()),
                    cond_ratio=float((crel_el[big] / cond[big]).max(initial=0.0)))
    print("FP32 refit covariance tails:", out)
    return out


def test_refit_covariance_clauses_admit_fp32_and_are_no_looser(refit_tails):
    """Each refit clause admits the worst FP32 build and is at most the
    tracklet clauses' margins (1.1x, 1.5x, 1.05x) beyond it."""
    assert all(t["n"] > 300000 for t in refit_tails.values())
    short = 1.0 - min(t["within_1e3"] for t in refit_tails.values())
    assert short <= 1.0 - parity.REFIT_MIN_COV_FRACTION <= 1.1 * short
    short_mid = 1.0 - min(t["within_1e2"] for t in refit_tails.values())
    assert short_mid <= 1.0 - parity.REFIT_MIN_COV_MID_FRACTION <= 1.5 * short_mid
    ratio = max(t["cond_ratio"] for t in refit_tails.values())
    assert ratio <= parity.REFIT_COV_COND_K <= 1.05 * ratio


# ----------------------------------------------------------------------------
# the chain fit's bulk covariance fractions (parity.CHAIN_*)

@pytest.fixture(scope="module")
def chain_tails(tmp_path_factory):
    """Covariance deviations of FP32 builds of the oracle's chain fit from its
    FP64 fit, over the chains the oracle merger forms on the 50-collision
    frame."""
    import synth
    from test_merge_oracle import merge_event
    tmp = tmp_path_factory.mktemp("fp32_chain")
    ev, o, r, unit, fr, lr, alpha, side, m = merge_event("pbpb_timeframe_50")
    heads, cf, cn, ch, cu = oracle.chains(m["next"], m["prev"], o["track_first_hit"], o["track_n_hits"],
                                          o["track_hits"], unit)
    k = float(np.float32(-np.float32(synth.KAPPA) * np.float32(ev.bz)))

    def run(lib):
        saved = (oracle._LIB, oracle._lib)
        if lib:
            oracle._LIB, oracle._lib = lib, None
        try:
            return oracle.refit_chains(cf, cn, ch, cu, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), alpha, k, P)
        finally:
            oracle._LIB, oracle._lib = saved

    c64 = run(None)
    out = {}
    for sym in (False, True):
        for fma in ((False, True) if _cpu_has_fma() else (False,)):
            c32 = run(_build(tmp, sym, fma))
            both = c64["ok"].astype(bool) & c32["ok"].astype(bool)
            oc = c64["cov"][both][:, DIAG]
            gc = c32["cov"][both][:, DIAG].astype(np.float32).astype(np.float64)
            crel = (np.abs(gc - oc) / np.abs(oc)).max(axis=1)
            out[(sym, fma)] = dict(n=int(both.sum()), within_1e3=float((crel <= parity.COV_RTOL).mean()),
                                   within_1e2=float((crel <= parity.COV_RTOL_MID).mean()),
                                   cov_max=float(crel.max()))
    print("FP32 chain covariance tails:", out)
    return out


def test_chain_covariance_fractions_admit_fp32_and_are_no_looser(chain_tails):
    assert all(t["n"] > 100000 for t in chain_tails.values())
    short = 1.0 - min(t["within_1e3"] for t in chain_tails.values())
    assert short <= 1.0 - parity.CHAIN_MIN_COV_FRACTION <= 1.1 * short
    short_mid = 1.0 - min(t["within_1e2"] for t in chain_tails.values())
    assert short_mid <= 1.0 - parity.CHAIN_MIN_COV_MID_FRACTION <= 1.5 * short_mid
    # the clause on every entry stays the refit's: the builds' worst lies under its floor
    assert max(t["cov_max"] for t in chain_tails.values()) <= parity.COV_RTOL_ALL

