"""Test-only numpy executor of an exported plan schedule (complex128).

It re-derives every index map from the exported variable lists with its own
pext, so a wrong mask, table or leaf value in the planner shows up as a wrong
amplitude when compared with the oracle.  Not a product path: the library has
no CPU execution at all.
"""
import numpy as np


def pext_vec(x: np.ndarray, mask: int) -> np.ndarray:
    out = np.zeros_like(x)
    k = 0
    for b in range(32):
        if (mask >> b) & 1:
            out |= ((x >> b) & 1) << k
            k += 1
    return out


def popcount(x: int) -> int:
    return bin(x).count("1")


def derived_masks(plan, steps, tens):
    """Masks recomputed from the kappa and variable lists of each step."""
    out = []
    for t, rec in enumerate(steps):
        nin, nk, rC = int(rec[1]), int(rec[2]), int(rec[3])
        kappa = plan.kappa(t)
        ovars = [int(v) for v in tens[rec[0], 4:4 + rC]]
        ivars = list(kappa) + ovars
        rI = len(ivars)
        ms = []
        for i in range(nin):
            tr = tens[rec[5 + i]]
            tv = [int(v) for v in tr[4:4 + tr[0]]]
            m = 0
            for j, v in enumerate(ivars):
                if v in tv:
                    m |= 1 << (rI - 1 - j)
            ms.append(m)
        out.append(ms)
    return out


def run(plan, slices, bitstrings=None):
    """Per-bitstring lists of slice values (prefactor applied)."""
    steps, tens = plan.export()
    info = plan.info()
    B = info["n_bitstrings"]
    pref = info["prefactor"]
    leaves = {}
    for t in range(tens.shape[0]):
        if tens[t, 1] == 0:
            leaves[t] = plan.leaf_values(t)
    res = []
    for b in (range(B) if bitstrings is None else bitstrings):
        vals = []
        for s in slices:
            env = {}
            for rec in steps:
                nin, nk, rC = int(rec[1]), int(rec[2]), int(rec[3])
                rI = nk + rC
                I = np.arange(1 << rI, dtype=np.int64)
                prod = np.ones(1 << rI, dtype=np.complex128)
                for i in range(nin):
                    tid = int(rec[5 + i])
                    mask = int(rec[13 + i]) & 0xFFFFFFFF
                    tr = tens[tid]
                    rank, kind, flags, sel = int(tr[0]), int(tr[1]), int(tr[2]), int(tr[3]) & 0xFFFFFFFF
                    if kind == 0:
                        nvar = 1 << popcount(sel)
                        arr = leaves[tid].reshape(-1, nvar, 1 << rank)
                        arr = arr[b if flags & 1 else 0, int(pext_vec(np.array([s]), sel)[0])]
                    else:
                        arr = env[tid]
                    prod = prod * arr[pext_vec(I, mask)]
                env[int(rec[0])] = prod.reshape(1 << nk, 1 << rC).sum(axis=0)
            vals.append(complex(env[int(steps[-1][0])][0]) * pref)
        res.append(vals)
    return res
