"""MI355X-native multi-morphology compartmental neuron simulator.

The simulation itself lives in a HIP shared library (``libmmhines.so``) behind
the C ABI declared in ``include/sim.h``; :mod:`paper_2005_06332_amd.sim` is a
thin ctypes binding over it and :mod:`paper_2005_06332_amd.workload` draws
seeded synthetic inputs. Importing the package loads nothing native.
"""
__all__ = ["workload", "sim"]
