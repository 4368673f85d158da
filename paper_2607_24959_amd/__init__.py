"""Batched regularised contact solves and their IFT derivative on MI355X (gfx950).

Layout of the package:
  synth      seeded synthetic instances (input construction only)
  _native    ctypes binding of libcs.so (include/cs.h)
  solver     torch-facing wrappers: forward, ift_vjp, unrolled_vjp
  build      compiles libcs.so in-tree for gfx950

Heavier modules (autograd function, batching, serving) import torch and the
native library lazily, so ``import paper_2607_24959_amd.synth`` stays cheap.
"""
__all__ = ["synth"]
