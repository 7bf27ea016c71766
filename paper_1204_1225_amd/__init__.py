"""Kirchhoff prestack migration (Eq. (1) of "Distributed computing of Seismic
Imaging Algorithms") on AMD Instinct MI355X: a HIP/gfx950 C-ABI library
(libkirchhoff.so, include/kirchhoff.h) with a thin PyTorch binding.

Submodules: survey (seeded synthetic inputs), ops (migrate / demigrate /
count / float64 reductions / tuning / batches), autograd (differentiable
operators), lsm (least-squares migration), build (compiles the library).
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["survey", "ops", "autograd", "lsm", "build"]
