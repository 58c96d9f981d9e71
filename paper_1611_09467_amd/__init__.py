"""pepsgo: MI355X-native per-sample evaluation of a finite open-boundary PEPS.

The compute path lives in the HIP shared library built from ``csrc/`` behind
the C-ABI declared in ``include/pepsgo.h``; ``pepsgo`` (this package's
``binding`` module) marshals arguments to it.  ``workloads`` holds the seeded
synthetic input generators.
"""
__all__ = ["workloads", "binding"]
