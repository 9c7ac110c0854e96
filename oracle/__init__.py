"""CPU oracle for the diffusive integer lattice gas with the flip operator.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or run anything in this package; the product
library (paper_2203_01380_amd) never does, and the two share no code.

  ilg_oracle.c  plain C step: Philox4x32-10 draws, chunked fixed-point
                binomials, flip -> collide -> stream, state hash.
  exact.py      exact big-integer tables, rational post-collision laws, the
                FP64 lattice Boltzmann / MRT limit and the paper's closed forms.
  oracle.py     ctypes front end and gcc build of ilg_oracle.c.

Parity unpinned: which sample path occurs (the assignment of Philox words to
binomial draws and of counters to nodes) is fixed only by this implementation's
own specification; it is checked as oracle-vs-GPU bit equality, while the law
of every sampled quantity is pinned against the paper and exact mathematics.
"""
