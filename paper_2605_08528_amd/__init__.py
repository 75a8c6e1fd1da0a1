"""MI355X-native batched driving-physics step (SceneFactory, arXiv 2605.08528).

The hot path lives in the HIP library ``libsf.so`` built from ``csrc/``; the
Python module :mod:`paper_2605_08528_amd.sf` marshals arguments to it.
:mod:`paper_2605_08528_amd.inputs` draws the seeded synthetic workloads.
Nothing is imported eagerly so that loading the input generator never needs
the native library.
"""
__all__ = ["inputs", "sf"]
