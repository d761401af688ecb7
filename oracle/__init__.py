"""FP64 CPU oracle of the mixing-graph method.  TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the HIP
library is checked against.  It is imported only by ``tests/``, by the smoke
check of the package entry file, and by the CPU-baseline leg of the benchmark.
The product path never imports, links or calls anything here, and nothing
here imports the product package: the two share only the seeded inputs of the
``synth`` module.

Contents (each function cites the passage of the paper it follows):
  processors.py  the processors of Sec. 3 and the tanh waveshaper
  console.py     node-by-node evaluation of a graph (Sec. 3 preamble, Sec. 4)
  loss.py        the A-weighted Mel MRSTFT loss and regularisers (Sec. 5.1)
  train.py       loss + gradients (autograd, plus the straight-through delay
                 rule of Sec. 3.7) and the Adam update
  prune.py       the batched brute-force pruning round

Parity status: every function is pinned by the tests in ``tests/`` marked
``not gpu`` (closed forms, special cases, brute force, finite differences),
except where a function's docstring says "parity unpinned".
"""
