"""pepsgo: MI355X-native per-sample evaluation of a finite open-boundary PEPS.

The compute path lives in the HIP shared library built from ``csrc/`` behind
the C-ABI declared in ``include/pepsgo.h``; ``binding`` marshals arguments to
it.  ``workloads`` holds the seeded synthetic input generators, ``workmodel``
the algorithmic flop counts the roofline uses, and ``protocols`` the
optimisation protocols of Sec. III (simple update to convergence, the D-ramp,
the gradient-step schedule) driven through the library's entry points.
"""
__all__ = ["workloads", "binding", "workmodel", "protocols"]
