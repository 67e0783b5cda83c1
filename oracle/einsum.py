"""np.einsum evaluated pairwise along a cached contraction order.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The order of the
pairwise contractions is chosen once per (subscripts, shapes) by numpy's greedy
path search; each pair is then evaluated by numpy (plain loops when small,
BLAS-backed tensordot when large).  Only the order is cached; the arithmetic
is numpy's.
"""
import numpy as np

_PLANS = {}
_SMALL = 1 << 17


def _plan(spec, ops):
    ins, out = spec.split("->")
    subs = ins.split(",")
    dims = {}
    for s, o in zip(subs, ops):
        dims.update(zip(s, o.shape))
    path = np.einsum_path(spec, *ops, optimize="greedy")[0][1:]
    steps = []
    cur = list(subs)
    for pair in path:
        pair = tuple(sorted(pair, reverse=True))
        taken = [cur.pop(k) for k in pair]
        rest = "".join(cur) + out
        keep = []
        for s in taken:
            for ch in s:
                if ch in rest and ch not in keep:
                    keep.append(ch)
        res = "".join(keep)
        loop = 1
        for ch in set("".join(taken)):
            loop *= dims[ch]
        steps.append((pair, ",".join(taken) + "->" + res, loop <= _SMALL))
        cur.append(res)
    return steps, cur[0] + "->" + out


def einsum(spec, *ops):
    ops = [np.asarray(o) for o in ops]
    if len(ops) == 1:
        return np.einsum(spec, *ops)
    key = (spec,) + tuple(o.shape for o in ops)
    plan = _PLANS.get(key)
    if plan is None:
        plan = _plan(spec, ops)
        _PLANS[key] = plan
    steps, final = plan
    cur = list(ops)
    for pair, sub, small in steps:
        taken = [cur.pop(k) for k in pair]
        r = np.einsum(sub, *taken) if small else np.einsum(sub, *taken, optimize=True)
        cur.append(r)
    return np.einsum(final, cur[0])
