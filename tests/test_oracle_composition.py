"""Pin of the oracle's cascade composition (Algorithm 1 and Algorithm 2).

The operators of the cascade are pinned one by one elsewhere (blur, restriction,
coarse PSF, smoothers, Pi, P, the linear prolongation, S and D).  Here the
complete cascade is rebuilt in Python from those pinned operator calls, in the
order the paper states it:

  Algorithm 2 (EECMG): levels 1 and 2 are smoothed from zero; then for each
  level l = 2 .. L-1 the next level starts from D(S(P(Pi(u_{l-1}, u_l)))) and
  is smoothed (Section 2; Pi and P in Section 3.2, S in Section 3.3, D in
  Section 4).
  Algorithm 1 (IECMG-L / IECMG-P): level 1 from zero; each next level starts
  from D(S(L u_l)) or D(S(P u_l)) and is smoothed (eq. 15 for L).

The rebuilt result must equal ``oracle.restore`` bit for bit, with the same
per-level iteration counts, stop reasons and final residuals.  A rebuilt
cascade with S and D swapped, or with Pi fed the wrong level pair, must not
match: those checks show that the pin can fail.
"""
import numpy as np
import pytest

import oracle
from paper_2311_03010_amd import synth


def _compose(g, psf, L, caps, smoother, cascade, stop_rule, delta, c=1.1, k=10.0, tau=0.2, pm_steps=1, smooth_h=1.0,
             eps=1e-14, order="PSD", pi_pair="prev"):
    sizes = oracle.level_sizes(*g.shape, L)
    # right-hand sides by injection (eq. 12-13) and the PSF pyramid (eq. 14)
    gs = [None] * L
    gs[L - 1] = np.array(g, dtype=np.float64)
    for l in range(L - 2, -1, -1):
        gs[l] = oracle.restrict(gs[l + 1], *sizes[l])
    psfs = [None] * L
    psfs[L - 1] = np.array(psf, dtype=np.float64)
    for l in range(L - 2, -1, -1):
        psfs[l] = oracle.coarse_psf(psfs[l + 1])
    smooth = oracle.cgls if smoother == 0 else oracle.mr
    cdelta = c * delta
    us = [None] * L
    iters, reasons, rms = [0] * L, [0] * L, [0.0] * L

    def run(l, u0):
        u, it, hist, why = smooth(gs[l], psfs[l], u0=u0, cap=caps[l], stop_rule=stop_rule, cdelta=cdelta, eps=eps)
        us[l], iters[l], reasons[l], rms[l] = u, it, why, float(hist[-1])

    n_start = (2 if L >= 2 else 1) if cascade == 0 else 1
    for l in range(n_start):
        run(l, np.zeros(sizes[l]))
    for lc in range(n_start, L):
        hc, wc = sizes[lc]
        if cascade == 0:
            ua = us[lc - 2] if pi_pair == "prev" else oracle.restrict(us[lc - 1], *sizes[lc - 2])
            v = oracle.prolong_quad(oracle.extrapolate(ua, us[lc - 1]), hc, wc)
        elif cascade == 1:
            v = oracle.prolong_linear(us[lc - 1], hc, wc)
        else:
            v = oracle.prolong_quad(us[lc - 1], hc, wc)
        if order == "PSD":
            v = oracle.local_smooth(v, smooth_h)
            for _ in range(pm_steps):
                v = oracle.pm_step(v, k, tau)
        else:  # D before S: a wrong order, for the negative check
            for _ in range(pm_steps):
                v = oracle.pm_step(v, k, tau)
            v = oracle.local_smooth(v, smooth_h)
        run(lc, v)
    return us[L - 1], {"iters": iters, "reason": reasons, "final_rms": rms}


def _case(L, H=97, W=83):
    # the 64^2 Gaussian recipe on a ragged grid, with as many levels as asked
    return synth.workload(1, H=H, W=W, n_levels=L)


@pytest.mark.parametrize("L", [3, 4, 5])
@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("stop_rule", [False, True])
@pytest.mark.parametrize("cascade", [0, 1, 2])
def test_restore_is_the_composition_of_the_pinned_operators(L, smoother, stop_rule, cascade):
    p = _case(L, H=97 if L < 5 else 131, W=83 if L < 5 else 140)
    caps = [3, 4, 5, 4, 3][:L]
    u_ref, st = oracle.restore(p.g_delta, p.psf, L, caps=caps, stop_rule=stop_rule, delta=p.delta,
                               smoother=smoother, cascade=cascade, guard_eps=1e-14)
    u, cs = _compose(p.g_delta, p.psf, L, caps, smoother, cascade, stop_rule, p.delta)
    np.testing.assert_array_equal(u, u_ref)
    assert cs["iters"] == st["iters"]
    assert cs["reason"] == st["reason"]
    assert cs["final_rms"] == st["final_rms"]


def test_composition_with_several_denoising_steps_and_scale():
    p = _case(4, H=90, W=101)
    kw = dict(k=5.0, tau=0.25, pm_steps=3, smooth_h=2.5)
    u_ref, _ = oracle.restore(p.g_delta, p.psf, 4, caps=[2, 3, 4, 3], stop_rule=False, delta=p.delta, **kw)
    u, _ = _compose(p.g_delta, p.psf, 4, [2, 3, 4, 3], 0, 0, False, p.delta, **kw)
    np.testing.assert_array_equal(u, u_ref)


@pytest.mark.parametrize("cascade", [0, 1, 2])
def test_wrong_stage_order_is_detected(cascade):
    # S and D swapped changes the result: the pin above would catch a cascade
    # that applied them in the other order
    p = _case(4)
    caps = [3, 4, 5, 4]
    u_ref, _ = oracle.restore(p.g_delta, p.psf, 4, caps=caps, stop_rule=False, delta=p.delta, cascade=cascade)
    u_bad, _ = _compose(p.g_delta, p.psf, 4, caps, 0, cascade, False, p.delta, order="DSP")
    assert np.linalg.norm(u_bad - u_ref) > 1e-6 * np.linalg.norm(u_ref)


def test_wrong_extrapolation_pair_is_detected():
    # Pi fed (restricted u_l, u_l) instead of (u_{l-1}, u_l): the corrections
    # vanish, so Pi reduces to the identity and the result changes
    p = _case(4)
    caps = [3, 4, 5, 4]
    u_ref, _ = oracle.restore(p.g_delta, p.psf, 4, caps=caps, stop_rule=False, delta=p.delta)
    u_bad, _ = _compose(p.g_delta, p.psf, 4, caps, 0, 0, False, p.delta, pi_pair="self")
    assert np.linalg.norm(u_bad - u_ref) > 1e-6 * np.linalg.norm(u_ref)
