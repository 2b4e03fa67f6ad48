"""Test harness helpers: matching storage DoFs of the HIP path to the oracle's
unique DoFs by their exact integer keys.  No arithmetic of the method here."""
from __future__ import annotations

import numpy as np


def _rows(v, w):
    return np.ascontiguousarray(np.hstack([v.astype(np.int64), w.astype(np.int64)]))


def storage_to_unique(gpu_keys, oracle_keys):
    """Index of each storage DoF's key among the oracle's unique keys."""
    gv, gw = gpu_keys
    ov, ow = oracle_keys
    g = _rows(gv, gw)
    o = _rows(ov, ow)
    both = np.vstack([o, g])
    _, first, inv = np.unique(both, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    no = o.shape[0]
    # every oracle key is unique, so the unique-set id of oracle row i maps back to i
    uid_of_set = np.full(len(first), -1, dtype=np.int64)
    uid_of_set[inv[:no]] = np.arange(no)
    m = uid_of_set[inv[no:]]
    if (m < 0).any():
        raise AssertionError("a storage key is missing from the oracle")
    return m


def copies_consistent(y_storage, s2u):
    """True iff all storage copies of every unique DoF hold bitwise-equal values."""
    order = np.argsort(s2u, kind="stable")
    su = s2u[order]
    yv = y_storage[order]
    same = su[1:] == su[:-1]
    return bool(np.all(yv[1:][same] == yv[:-1][same]))


def rel_err_max(a, b):
    """||a - b||_inf / ||b||_inf."""
    d = np.abs(np.asarray(a) - np.asarray(b)).max()
    s = np.abs(np.asarray(b)).max()
    return d / s if s > 0 else d
