"""Plain FP64 CPU oracle of the consistent SDF interpolation method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library: it is a slow, obviously correct restatement of the
paper's definitions, written in float64 NumPy (the paper performs all
intersection and containment checks in double precision, Appendix B).

Modules (each function cites the passage it follows):
  common   tolerances, kind codes, flag bits, the single covered predicate
  bounds   pairwise cone bounds lo/hi with argmax/argmin (Sec. 4.3)
  spheres  caps, circle arcs, exact uncovered-point search on a sphere
           (Prop. 1 (ii); the U/D candidates of Def. 1)
  rmin     minimum valid radius (Prop. 2 proof, Corollary 1, Sec. 6)
  order    covered-area ratios and the flood-fill refinement order (Sec. 4.2)
  greedy   greedy sequential interpolation (Sec. 3.3 + Sec. 4)
  certify  Prop. 1 certificate of a final sample set
  repair   pseudo-SDF repair (Sec. 6)
  adjoint  reverse sweep of d(sum of values)/d(inputs) over active parents
  tiny     paper-exact tier for tiny inputs: every Def. 1 grow-to point, the
           Sec. 3.3 scoring rule and Prop. 1 checked on the whole set
"""
