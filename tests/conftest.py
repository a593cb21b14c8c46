import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@functools.lru_cache(maxsize=None)
def cached_event(name, seed=None):
    import synth
    fn = synth.WORKLOADS[name]
    return fn() if seed is None else fn(seed)


@functools.lru_cache(maxsize=None)
def cached_oracle(name, seed=None, fragile_eps=0.05):
    import oracle
    from paper_2106_03636_amd.params import DEFAULT_PARAMS
    ev = cached_event(name, seed)
    return oracle.run_event(ev, DEFAULT_PARAMS, fragile_eps=fragile_eps)
