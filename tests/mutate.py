"""Planted mistakes for oracle modules (test helper, CPU only).

``mutated(module, old, new)`` returns a fresh copy of an oracle module whose
source has the text ``old`` replaced by ``new`` (exactly once).  A test
swaps the copy in for the original with ``monkeypatch`` and asserts that the
pins of that module then fail: a pin that a plausible slip cannot fail pins
nothing.
"""
from __future__ import annotations

import importlib.util
import inspect
import sys
import types


def mutated(module: types.ModuleType, old: str, new: str) -> types.ModuleType:
    src = inspect.getsource(module)
    n = src.count(old)
    if n != 1:
        raise AssertionError(f"mutation anchor {old!r} occurs {n} times in {module.__name__}")
    spec = importlib.util.spec_from_loader(module.__name__ + "_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = module.__package__
    mod.__file__ = module.__file__
    sys.modules[spec.name] = mod
    try:
        exec(compile(src.replace(old, new), module.__file__, "exec"), mod.__dict__)
    finally:
        sys.modules.pop(spec.name, None)
    return mod
