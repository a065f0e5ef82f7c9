"""MI355X-native Particles-on-Demand (PonD) finite-volume time step.

The product is the HIP library ``libpond.so`` behind the C interface declared
in ``include/pond.h``; ``paper_2302_00310_amd.pond`` is its thin Python
binding.  Importing this package loads nothing by itself.
"""
