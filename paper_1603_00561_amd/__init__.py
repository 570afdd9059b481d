"""MI355X-native DF-DSRG-MRPT2 pair-energy library (terms F1-F3).

The compute path lives in the HIP shared library ``libdsrgdf.so`` built from
``csrc/``; :mod:`.binding` loads it. Importing this package does not load the
library, so the seeded workload generator can be used on machines without it.
"""

__all__ = ["workloads", "binding"]


def __getattr__(name):
    if name == "binding":
        from . import binding
        return binding
    if name == "workloads":
        from . import workloads
        return workloads
    raise AttributeError(name)
