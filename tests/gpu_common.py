"""Shared helpers of the GPU parity tests (inputs from the seeded generator,
expected values from the oracle only)."""
import numpy as np
import torch

import oracle
from paper_1911_02366_amd import Plan

DEV = "cuda"


def to_np(t):
    return t.detach().cpu().numpy()


def oracle_arrays(case):
    return dict(order=case.order, c_ptr=case.c_ptr, c_node=case.c_node, bb_rowptr=case.bb_rowptr,
                bb_col=case.bb_col, bb_val=to_np(case.bb_val), aii=to_np(case.aii),
                aib=to_np(case.aib), abi=to_np(case.abi), b=to_np(case.rhs))


def oracle_matrix(d):
    return oracle.assemble_global(d["order"], d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"],
                                  d["bb_val"], d["aii"], d["aib"], d["abi"])


def device_case(case):
    return dict(aii=case.aii.to(DEV).contiguous(), aib=case.aib.to(DEV).contiguous(),
                abi=case.abi.to(DEV).contiguous(), bb_val=case.bb_val.to(DEV).contiguous(),
                b=case.rhs.to(DEV).contiguous())


def make_plan(case, dev, precision="fp64"):
    plan = Plan.from_structure(case.structure())
    plan.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    plan.factor(precision)
    plan.condense()
    return plan


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def fold_matrices(case, elems=None):
    """F_e: the A_bb blocks the library folds into element e's stored Schur block.

    Rule (documented in the C header): block (g, h) goes to the element that owns
    boundary node g when both g and h are in its coupling set, else to the
    lowest-numbered element whose coupling set holds both; otherwise it stays in
    the remainder.  Returns {e: F_e} for the requested elements (default all)."""
    n_e = case.n_elem
    orders = np.asarray(case.order)
    bnode_off = np.concatenate([[0], np.cumsum((orders + 1) ** 3 - (orders - 1) ** 3)])
    elems = range(n_e) if elems is None else elems
    c_sets = lambda e: case.c_node[case.c_ptr[e]:case.c_ptr[e + 1]]
    pos_cache = {}

    def pos(e):
        if e not in pos_cache:
            pos_cache[e] = {int(g): i for i, g in enumerate(c_sets(e))}
        return pos_cache[e]

    holders = {}
    for e in range(n_e):
        for g in c_sets(e):
            holders.setdefault(int(g), []).append(e)
    vals = to_np(case.bb_val).reshape(-1, 5, 5)
    out = {}
    for e in elems:
        nc = 5 * int(case.c_ptr[e + 1] - case.c_ptr[e])
        f = np.zeros((nc, nc))
        pe = pos(e)
        for g in c_sets(e):
            g = int(g)
            owner = int(np.searchsorted(bnode_off, g, side="right") - 1)
            cands = sorted(holders[g], key=lambda x: (x != owner, x))
            for t in range(case.bb_rowptr[g], case.bb_rowptr[g + 1]):
                h = int(case.bb_col[t])
                if h not in pe:
                    continue
                chosen = next(x for x in cands if h in pos(x))
                if chosen == e:
                    pg, ph = pe[g], pe[h]
                    f[5 * pg:5 * pg + 5, 5 * ph:5 * ph + 5] += vals[t]
        out[e] = f
    return out
