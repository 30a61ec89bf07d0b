"""MI355X-native He-Luo MRT lattice Boltzmann step with the Yu and Chai strain-rate
formulas (arXiv 1704.07559), behind the C ABI of include/lbm.h.

Importing the package loads nothing; ``paper_1704_07559_amd.capi`` loads liblbm.so (and
raises if it has not been built), ``paper_1704_07559_amd.lbm`` adds a torch-buffer wrapper,
``autograd`` the strain-loss gradient, ``checkpoint`` file checkpoints and a guarded run loop.
"""
__all__ = ["capi", "lbm", "autograd", "checkpoint", "build"]
