"""CPU oracle for PBN simulation (TEST INFRASTRUCTURE ONLY).

This package is the plain, slow reference that the GPU library is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library's product path never does, and nothing
here imports the library.  Everything is written from the paper
(Mizera, Pang, Yuan: "Fast Simulation of Probabilistic Boolean Networks",
arXiv:1605.00854) and from the published definitions of the generators it
uses; the two implementations share only the seeded input generators.

Modules
  philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  contract   random-number keying, integer quantisation, initial state
  simulate   trajectories of the *unreduced, ungrouped* network (Eq. 1, Sec. 2.2)
  exact      2^n transition matrix (Eq. 1) and its steady state, n <= 12
  structure  leaf nodes (Def. 1), Eq. 2 bound, greedy partition (Alg. 3),
             Partition (Alg. 4), single-predictor grouping (Sec. 3.3),
             combined predictor functions (Sec. 3.3)
  stats      estimators: trajectory means, batch means, two-state chain figures
  skart      the Skart stopping rule (skewness- and correlation-adjusted batch means)
"""
