"""MI355X-native DF-DSRG-MRPT2 pair-energy library (terms F1-F3).

The compute path lives in the HIP shared library ``libdsrgdf.so`` built from
``csrc/``; :mod:`paper_1603_00561_amd.binding` loads it and
:mod:`paper_1603_00561_amd.autograd` wraps it for torch. Importing this
package itself loads nothing, so the seeded workload generator
(:mod:`paper_1603_00561_amd.workloads`) works where the library is absent.
"""
