"""Shared checks of the GPU tests (no test functions here).

site_errors: the relative L2 error over sampled output sites, printed with the
largest relative error of any single site (each site's 12 complex components
against the reference site's norm), so that a small whole-field figure cannot
hide one bad site.

check_true_residual: a solution's FP64 true relative residual ||b - D x|| / ||b||
recomputed by the oracle on the host must meet the tolerance and agree with the
residual the library itself reports (info["true_rel_residual"]), so that the
two independent evaluations pin each other.  They round differently: each
entry of b - D x carries an FP64 rounding error of about 1e-16 ||x|| per term,
so at residuals near 1e-12 the two relative residuals differ by a few 1e-18
(a few 1e-6 of the value on the smallest lattices, where little averages
out); the check allows 1e-6 relative plus 1e-15 absolute, far below what a
dropped term or a wrong sign would change.
"""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def site_errors(out_sites, ref_sites, label=""):
    """(relative L2 error, largest per-site relative error) of (n, 4, 3) arrays."""
    out_sites = np.asarray(out_sites).reshape(len(ref_sites), -1)
    ref_sites = np.asarray(ref_sites).reshape(len(ref_sites), -1)
    d = np.linalg.norm(out_sites - ref_sites, axis=1)
    r = np.linalg.norm(ref_sites, axis=1)
    l2 = float(np.linalg.norm(d) / np.linalg.norm(r))
    per_site = float(np.max(d / np.where(r > 0, r, 1.0)))
    say("%s%d sites: rel L2 err %.3e, max per-site rel err %.3e" % (label + " " if label else "", len(ref_sites),
                                                                   l2, per_site))
    return l2, per_site


def rel(a, b):
    """Whole-field relative L2 error of a against b; for spinor fields (last axes
    4 x 3) the largest per-site relative error (each site's 12 components against
    the reference site's norm, sites where the reference is zero left out) is
    printed beside it."""
    a = np.asarray(a)
    b = np.asarray(b)
    e = float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    if a.ndim >= 2 and a.shape[-2:] == (4, 3):
        d = np.linalg.norm((a - b).reshape(-1, 12), axis=1)
        r = np.linalg.norm(b.reshape(-1, 12), axis=1)
        m = r > 0
        say("rel L2 err %.3e, max per-site rel err %.3e over %d sites" % (e, float(np.max(d[m] / r[m])), int(m.sum())))
    return e


def check_true_residual(U, kappa, csw, b, x, info, tol, agree=1e-6):
    """Oracle residual of x below tol, and equal to the library's own to `agree`
    (relative) plus 1e-15.  Returns the oracle's relative residual."""
    r, bn = oracle.residual(U, kappa, csw, b, x)
    rr = r / bn
    lib = info["true_rel_residual"]
    say("true rel residual: oracle %.6e, library %.6e" % (rr, lib))
    assert rr < tol, (rr, tol)
    assert abs(rr - lib) <= agree * rr + 1e-15, (rr, lib)
    return rr
