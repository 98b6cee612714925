"""CPU FP64 oracles of the hierarchical method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
GPU library never imports, links or calls it, and the two share no code.

* ``oracle.hier``  plain recursive C implementation (tree, Algorithm 1-3).
* ``oracle.dense`` numpy/LAPACK dense Z, projector and complement basis.
* ``oracle.bd``    the constrained Brownian-dynamics solve of Eqs. 1.5-1.6,
  dense, in ``oracle.hier``'s basis (small systems).
"""
