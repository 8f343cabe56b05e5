"""Field-by-field comparison of solver vectors (test helper, no arithmetic of
the method).

A KKT iterate stacks fields of very different size: at alpha = 1e-8 the
multiplier lambda of eq. mp2 is about 1e-5 of the state y, so one norm over
the whole vector would let lambda (and the control u = alpha^-1 lambda,
section 1) drift far above the stated tolerance.  Every comparison here is
therefore made per field, as max |got - ref| / max |ref| over that field."""
import numpy as np

POISSON_FIELDS = ("y", "lambda")
STOKES_FIELDS = ("v1", "v2", "p", "lambda1", "lambda2", "mu")


def stokes_sizes(level):
    n = 1 << level
    m = 2 * n - 1
    nv, npv = m * m, (n + 1) * (n + 1)
    return [nv, nv, npv, nv, nv, npv]


def split(x, problem="poisson", level=None):
    """{field name: view} of a Poisson vector [y | lambda] or a Stokes vector
    [v1 | v2 | p | lambda1 | lambda2 | mu]."""
    x = np.asarray(x)
    if problem == "poisson":
        V = x.size // 2
        return {"y": x[:V], "lambda": x[V:]}
    sizes = stokes_sizes(level)
    assert sum(sizes) == x.size, (sum(sizes), x.size)
    out, at = {}, 0
    for name, k in zip(STOKES_FIELDS, sizes):
        out[name] = x[at:at + k]
        at += k
    return out


def field_errors(got, ref, problem="poisson", level=None, alpha=None):
    """max |got - ref| / max |ref| per field; with alpha also for the control
    u = lambda / alpha (Poisson "u", Stokes "u1", "u2")."""
    g, r = split(got, problem, level), split(ref, problem, level)
    err = {}
    for k in r:
        err[k] = float(np.abs(g[k] - r[k]).max() / max(np.abs(r[k]).max(), 1e-300))
    if alpha is not None:
        pairs = [("u", "lambda")] if problem == "poisson" else [("u1", "lambda1"), ("u2", "lambda2")]
        for u, lam in pairs:
            gu, ru = g[lam] / alpha, r[lam] / alpha
            err[u] = float(np.abs(gu - ru).max() / max(np.abs(ru).max(), 1e-300))
    return err


def assert_fields(got, ref, tol, problem="poisson", level=None, alpha=None, what=""):
    err = field_errors(got, ref, problem, level, alpha)
    bad = {k: v for k, v in err.items() if not v <= tol}
    assert not bad, (what, tol, err)
    return err
