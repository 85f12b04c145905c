"""MI355X-native hot path of the sum-over-Cliffords simulator of Bravyi et al.,
"Simulation of quantum circuits by low-rank stabilizer decompositions"
(arXiv:1808.00128).

The compute path is the HIP library ``libchsim.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/chsim.h``; ``binding`` is its thin
ctypes front end.  ``workloads`` draws seeded synthetic inputs.
"""
import importlib

__all__ = ["binding", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
