"""Shared test helpers: translate a seeded Problem into oracle parameters and
compute the error measures used by the parity tests."""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle import Oracle, OracleParams


def oracle_for(prob, shifted: bool = True, threads: int = 1) -> Oracle:
    kw = dataclasses.asdict(prob)
    return Oracle(OracleParams(shifted=shifted, **kw), threads=threads)


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """sqrt(sum |a - ref|^2 / sum |ref|^2) over all nodes and components."""
    num = float(((a - ref) ** 2).sum())
    den = float((ref ** 2).sum())
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def eps_paper(a: np.ndarray, ref: np.ndarray) -> float:
    """sum_n |a - ref| / sum_n |ref| with pointwise Euclidean norms over the
    leading component axis (the paper's error measure)."""
    num = np.sqrt(((a - ref) ** 2).sum(axis=0)).sum()
    den = np.sqrt((ref ** 2).sum(axis=0)).sum()
    return float(num / den)
