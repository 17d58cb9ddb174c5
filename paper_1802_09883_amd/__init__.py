"""Reproducible floating-point GroupBy-SUM (repro<T,L>) on AMD MI355X.

Kernels and the C interface live in ``csrc/`` (built into ``librepro.so``);
``paper_1802_09883_amd.api`` holds the PyTorch-facing wrappers.  Importing the
package does not load the library; the first call does, and fails loudly if
it is missing.
"""
from ._lib import ERR_KEY, ERR_NONFINITE, ERR_RANGE  # noqa: F401
