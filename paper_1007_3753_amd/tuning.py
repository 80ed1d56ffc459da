"""JSON cache of tuned launch shapes (the split-K table of the DALM iteration
product), keyed by device architecture, problem shape, batch capacity and
arithmetic.  ``tune(plan)`` runs the library's autotuner
(l1_alm_tune_ksplit) and records the result; ``apply(plan)`` installs a
cached table if one exists for the plan's key."""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "ksplit_cache.json")


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def key(plan):
    return (f"{_arch()}|{plan.structure}|{plan.problem}|m{plan.m}|n{plan.n_dict}|"
            f"batch{plan.max_batch}|{plan.precision}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(plan, path=CACHE):
    entry = _load(path).get(key(plan))
    return None if entry is None else list(entry["ksplit"])


def apply(plan, path=CACHE):
    """Install the cached table for this plan; returns it, or None."""
    table = lookup(plan, path)
    if table is not None:
        plan.set_ksplit(table)
    return table


def tune(plan, iters=256, path=CACHE):
    """Tune this plan's split-K table, install it and record it in the cache
    at ``path``; returns the table."""
    table = plan.tune_ksplit(iters)
    data = _load(path)
    data[key(plan)] = {"ksplit": table, "iters": int(iters)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    return table
