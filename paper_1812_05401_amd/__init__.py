"""MI355X-native volume-penalization lattice Boltzmann (VP-LBM) step, arXiv:1812.05401.

The compute path is the HIP library ``libvplbm.so`` behind the C ABI in ``include/vplbm.h``;
``binding`` marshals arguments to it.  ``inputs`` draws seeded synthetic workloads.
"""
__all__ = ["inputs", "binding"]
