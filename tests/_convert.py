"""Test-side helpers: build matching problem descriptors for the HIP path and the oracle."""
import numpy as np

from oracle import scheme as OS


def problems(device="cuda", mu=None, gvec=None, **kw):
    """Returns (hip Problem, oracle Problem) with identical settings; mu / gvec given as numpy."""
    import torch
    import paper_2510_02635_amd as F
    hip_kw = dict(kw)
    if mu is not None:
        hip_kw["mu"] = torch.as_tensor(mu, dtype=torch.float64, device=device)
    if gvec is not None:
        hip_kw["gvec"] = torch.as_tensor(gvec, dtype=torch.float64, device=device)
    hp = F.Problem(**hip_kw)
    okw = {k: v for k, v in kw.items() if k in OS.Problem.__dataclass_fields__}
    op = OS.Problem(mu=None if mu is None else np.asarray(mu, dtype=np.float64),
                    gvec=None if gvec is None else np.asarray(gvec, dtype=np.float64), **okw)
    return hp, op


def rel_err(a, b):
    """The larger of the norm-wise relative error |a - b| / |b| and the element-wise one,
    max_i |a_i - b_i| / max_i |b_i|: a tolerance on it bounds every element, not only the norm."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    norm = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    elem = float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
    return max(norm, elem)
