"""Force-error metrics and gates shared by the GPU parity tests.

Two figures at identical positions (never along diverging trajectories):

* eps_F = ||F - F_ref||_2 / ||F_ref||_2 over the 3N vector: the relative
  force error; gates 1e-12 (FP64) and 1e-5 (mixed).
* the per-atom figure max_i |F_i - F_ref,i| / rms_i |F_ref,i|: catches a
  single wrong atom (a dropped pair, a wrong wall sum) that the norm would
  average away at large N.  Gates 1e-11 (FP64) and 1e-4 (mixed): rounding
  alone stays an order of magnitude below them (FP32 pair terms on cell-local
  coordinates carry a relative error of a few 1e-7 per pair, about 1e-5 of
  the largest pair force at a 0.9 sigma contact, which is at most a few times
  the rms force), while a single missing pair changes an atom's force by at
  least the force at the cutoff, 0.039 eps/sigma, i.e. more than 1e-3 of the
  rms force of every workload here.
"""
import numpy as np

TOL_F = {"fp64": 1e-12, "mixed": 1e-5}
TOL_ATOM = {"fp64": 1e-11, "mixed": 1e-4}


def force_errors(F, F_ref):
    """(eps_F, per-atom error / rms force) of F against F_ref, both [n][d]."""
    F_ref = np.asarray(F_ref, dtype=np.float64)
    d = F_ref.shape[-1] if F_ref.ndim > 1 else 3
    F = np.asarray(F, dtype=np.float64).reshape(-1, d)
    F_ref = F_ref.reshape(-1, d)
    d = F - F_ref
    nref = float(np.linalg.norm(F_ref))
    rms = float(np.sqrt(np.mean(np.sum(F_ref * F_ref, axis=1)))) if F_ref.size else 0.0
    if nref == 0.0:
        e = 0.0 if not np.any(d) else float("inf")
        return e, e
    return float(np.linalg.norm(d) / nref), float(np.sqrt(np.sum(d * d, axis=1)).max() / rms)


def check_forces(F, F_ref, prec, factor=1.0, what=""):
    """Assert both gates (each times `factor`); returns the two figures."""
    eps, atom = force_errors(F, F_ref)
    print("force error %s [%s]: eps_F %.3e, per-atom/rms %.3e" % (what, prec, eps, atom), flush=True)
    assert eps <= TOL_F[prec] * factor, (what, prec, "eps_F", eps)
    assert atom <= TOL_ATOM[prec] * factor, (what, prec, "per-atom", atom)
    return eps, atom
