"""Helpers shared by the GPU parity tests: tolerances and tie certification.

Per-region parity (same region list): |V_gpu - V_cpu| <= 1e-12 |V_cpu| +
floorV and the same for E with floorE, where the floors are the oracle's
256-ulp bounds on the rounding of the cancelling weighted sums. The split
axis must be equal unless the oracle certifies that the two axes are tied
up to rounding (the GPU's axis lies within the rounding slack of the tie
band's edge and no surely-tied axis beats it in the tie order).
"""
import numpy as np

REL = 1e-12


def certify_axis(D, w, kg, floorD):
    """True if axis kg is a legitimate choice for fourth differences D (one
    region) given their rounding: see the module docstring."""
    dmax = D.max()
    slack = 1e-12 * dmax + floorD
    edge = dmax * (1 - 1e-10) - floorD
    if D[kg] < edge - slack:
        return False
    for j in range(len(D)):
        if j == kg or D[j] < edge + slack:
            continue
        if w[j] > w[kg] or (w[j] == w[kg] and j < kg):
            return False
    return True


def assert_region_parity(ref, lo, w, V, E, K, rel=REL, max_uncertified=0):
    """ref: oracle.RegionEval; lo/w: [d, n] numpy; V/E/K: numpy from GPU."""
    dV = np.abs(V - ref.V)
    okV = dV <= rel * np.abs(ref.V) + ref.floorV
    assert okV.all(), ("V", np.flatnonzero(~okV)[:10], dV[~okV][:5], ref.V[~okV][:5])
    dE = np.abs(E - ref.E)
    okE = dE <= rel * np.abs(ref.E) + ref.floorE
    assert okE.all(), ("E", np.flatnonzero(~okE)[:10], dE[~okE][:5], ref.E[~okE][:5],
                       ref.floorE[~okE][:5])
    bad = np.flatnonzero(K != ref.K)
    uncert = [i for i in bad if not certify_axis(ref.D[i], w[:, i], int(K[i]), ref.floorD[i])]
    assert len(uncert) <= max_uncertified, ("K", uncert[:10], K[uncert[:10]], ref.K[uncert[:10]])
    return len(bad)


def rel_close(a, b, rel):
    return abs(a - b) <= rel * max(abs(a), abs(b))


def check_free_run(r, exact, tau, allow_no_active=False):
    """A free run against the closed form. OK: the estimate is within tau of
    the integral and the reported error within tau of the estimate. With
    allow_no_active (runs under the P_max rule of Section 3.5.3, whose
    threshold searches may commit so much error to finished regions that
    every region finishes while the summed error is still just above
    tau |v|) a NO_ACTIVE end is accepted as an honest near miss: the
    reported error exceeds tau |v| (the status is right) by less than a
    factor of 3, and the estimate lies within 3 tau of the integral. Such a
    run has not met its tolerance, so the estimate may miss tau itself (a
    d=6 corner peak of the batched workload ends 2.3 tau from its integral
    with a reported error of 1.1 tau)."""
    name = getattr(r, "status_name", None)
    true_err = abs(r.estimate - exact)
    if name == "NO_ACTIVE" and allow_no_active:
        assert tau * abs(r.estimate) < r.error <= 3 * tau * abs(r.estimate), r
        assert true_err <= 3 * tau * abs(exact), (r, exact)
        return
    assert name == "OK", r
    assert true_err <= tau * abs(exact), (r, exact)
    assert r.error <= tau * abs(r.estimate), r


def search_diff(rep):
    """The replay's record of the first threshold search whose outcome
    differs (iteration, the trace's ok / trials / t, the oracle's), for
    assertion messages."""
    keys = ("search_hard_it", "gpu_ok", "gpu_trials", "gpu_t", "cpu_ok",
            "cpu_trials", "cpu_t")
    return {k: rep[k] for k in keys if k in rep} if rep.get("search_hard") else {}
