"""MI355X-native two-component D2Q9 Shan-Chen lattice Boltzmann step.

The compute path lives in the HIP library ``liblb.so`` (sources in ``csrc/``,
C-ABI declared in ``include/lb.h``).  ``lb`` is its thin ctypes binding;
``inputs`` draws seeded initial densities.  Importing this package does not
load the library; ``paper_2101_04847_amd.lb`` does, and fails loudly if it is
missing.
"""
__all__ = ["inputs", "lb", "build"]
