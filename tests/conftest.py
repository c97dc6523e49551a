import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


_CASES = {}


def get_case(name, **kw):
    from ns_inputs import build
    key = (name, tuple(sorted(kw.items())))
    if key not in _CASES:
        _CASES[key] = build(name, **kw)
    return _CASES[key]


_ASM = {}


def get_assembled(name, **kw):
    from oracle import discretization as dz
    key = (name, tuple(sorted(kw.items())))
    if key not in _ASM:
        _ASM[key] = dz.assemble(get_case(name, **kw))
    return _ASM[key]
