"""Exhaustive search for tiny instances -- TEST INFRASTRUCTURE ONLY.

Evaluates the objective of the WCSP definition (Sec. 2, Eq. for sigma*) on
every complete assignment: the cost of an assignment is the sum of every
function's entry, infinity absorbing (R6: saturating at INT32_MAX), and the
optimum is the minimum.  For belief networks it evaluates the MPE objective
(Sec. 3) as a product of probabilities, without any logarithm, so that it
does not share the -ln p reduction with the eliminator it checks.
"""
from __future__ import annotations

import numpy as np

INF_I32 = 2**31 - 1


def all_assignments(domains) -> np.ndarray:
    """Every complete assignment, one row each, variable 0 most significant."""
    domains = [int(d) for d in domains]
    total = int(np.prod(domains)) if domains else 1
    if total > 5_000_000:
        raise ValueError("instance too large for exhaustive search")
    grids = np.indices(domains).reshape(len(domains), -1).T if domains else np.zeros((1, 0), np.int64)
    return grids.astype(np.int64)


def entry_index(domains, scope, sigma: np.ndarray) -> np.ndarray:
    """Row of a table over `scope` (as listed, first variable most
    significant) selected by each assignment in sigma."""
    idx = np.zeros(sigma.shape[0], np.int64)
    for v in scope:
        idx = idx * int(domains[int(v)]) + sigma[:, int(v)]
    return idx


def costs(inst, sigma: np.ndarray) -> np.ndarray:
    """Cost of every assignment (rows of sigma), saturating at INF_I32."""
    tot = np.zeros(sigma.shape[0], np.int64)
    for s, t in zip(inst.scopes, inst.tables):
        tot += np.asarray(t, np.int64)[entry_index(inst.domains, s, sigma)]
        np.minimum(tot, INF_I32, out=tot)
    return tot


def optimum(inst):
    """(min cost, one minimising assignment) of an int32 WCSP."""
    sigma = all_assignments(inst.domains)
    c = costs(inst, sigma)
    i = int(np.argmin(c))
    return int(c[i]), sigma[i]


def cost_of(inst, assignment) -> int:
    return int(costs(inst, np.asarray(assignment, np.int64)[None, :])[0])


def mpe(inst):
    """(max probability, maximising assignment) of a belief network."""
    sigma = all_assignments(inst.domains)
    prob = np.ones(sigma.shape[0], np.float64)
    for s, t in zip(inst.scopes, inst.tables):
        prob *= np.asarray(t, np.float64)[entry_index(inst.domains, s, sigma)]
    i = int(np.argmax(prob))
    return float(prob[i]), sigma[i]


def log_partition(inst) -> float:
    """-ln Z, Z = sum over every assignment of the product of the functions'
    factors: probabilities as given (prob_f64), exp(-cost) for double costs
    (cost_f64).  The sum is taken in probability space; the logarithm only
    at the end."""
    sigma = all_assignments(inst.domains)
    w = np.ones(sigma.shape[0], np.float64)
    for s, t in zip(inst.scopes, inst.tables):
        e = np.asarray(t, np.float64)[entry_index(inst.domains, s, sigma)]
        w *= e if inst.kind == "prob_f64" else np.exp(-e)
    with np.errstate(divide="ignore"):
        return float(-np.log(w.sum()))
