"""CPU oracle for the Generic Join hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import or run anything in this package.  It shares no code
with the GPU library (``paper_2502_06715_amd``): the only common module is the
seeded input generator ``paper_2502_06715_amd.inputs``, which holds none of
the join method's arithmetic.

Contents
  gj.c / oracle.py   Generic Join over sorted int64 tuple arrays (C, OpenMP),
                     with range predicates, output digest and work counter
  textbook.c         classical triangle / 4-clique counters (pins for the oracle)
  brute.py           brute-force enumeration of tiny instances (pins)
  coco.py            the CoCo levels and partition histograms by definition
  rewrite.py         the lifted-intersection rewriting, executed literally
  cells.py           HyperCube cells: Generic Join per cell, with the partition
                     checks (disjoint cell outputs whose union is Q(D))
"""
