"""Error measures shared by the GPU parity tests.

Every comparison with the oracle reports two numbers and gates both:
  rel  = ||got - want||_2 / ||want||_2      (relative L2 over the output)
  elem = max |got - want| / max |want|      (element by element, against the
                                             output's largest magnitude)
FP32 storage: the L2 gate of the operator and an element-wise gate of the
same size.  BF16 output storage: the L2 gate 2e-3 and an element-wise gate
of 2^-8 (+1%), half a BF16 unit in the last place relative to the value,
which bounds the output rounding of every element.
"""
import sys

import numpy as np

BF16_ELEM = 2.0 ** -8 * 1.01


def errs(got, want):
    g = np.asarray(got, dtype=np.float64).ravel()
    w = np.asarray(want, dtype=np.float64).ravel()
    d = g - w
    return (float(np.linalg.norm(d) / np.linalg.norm(w)),
            float(np.max(np.abs(d)) / np.max(np.abs(w))))


def check(tag, got, want, l2, elem=None):
    """Print both measures for `tag`, then assert rel <= l2 and
    elem <= (elem or l2).  Returns (rel, elem)."""
    r, m = errs(got, want)
    e = l2 if elem is None else elem
    print(f"  {tag}: rel L2 {r:.3e} (gate {l2:.1e})  max|d|/max|ref| {m:.3e} (gate {e:.1e})",
          flush=True)
    sys.stdout.flush()
    assert r <= l2, (tag, r, l2)
    assert m <= e, (tag, m, e)
    return r, m
