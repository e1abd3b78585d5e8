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
