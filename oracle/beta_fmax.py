"""Print the maximum of the oracle's unnormalised allowed beta shape (E0 = 18600 eV, Z = 2).

The rejection sampler needs an upper bound f_max of the shape; the workload module
stores a literal with 1 % headroom above the value printed here.  Calls only the oracle.
"""
import numpy as np

import oracle


def shape_max(e0: float = 18600.0, z: float = 2.0, n: int = 200001):
    es = np.linspace(0.0, e0, n)[1:-1]
    f = np.array([oracle.beta_shape(e, e0, z) for e in es])
    i = int(np.argmax(f))
    lo, hi = es[max(i - 1, 0)], es[min(i + 1, len(es) - 1)]
    fine = np.linspace(lo, hi, 20001)
    ff = np.array([oracle.beta_shape(e, e0, z) for e in fine])
    j = int(np.argmax(ff))
    return float(ff[j]), float(fine[j])


if __name__ == "__main__":
    fm, em = shape_max()
    print(f"max of the allowed beta shape: {fm:.6e} at E = {em:.3f} eV")
