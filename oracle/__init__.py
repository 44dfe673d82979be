"""CPU oracle for the baryon-baryon correlators (FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product (``paper_1510_00903_amd``) never imports it, and it never
imports the product: the two share no code, headers or tables.  Only the seeded
input generator ``synth`` feeds both.

Contents
  operators.py  gamma matrices, C gamma_5, the baryon fields and the 52 channels
                (Sec. 2 and Sec. 4 of the paper).
  wick.c/.py    O-W: the plain definition -- Wick's theorem as a signed sum over
                flavour-preserving bijections, and a direct O(V^2) sum over X.
  brute.py      O-0: literal 6x6 propagator determinants summed over every
                nonzero tensor index, for tiny lattices (pins O-W).
  grassmann.py  Wick contraction of Grassmann strings by explicit pairing
                (pins the determinant sign convention).
  unified.py    O-U: the same sum with the source-tensor and sigma sums folded
                into weights first and the X-sum done by a library FFT (the idea
                of the unified-contraction cross-check of Sec. 6).
  postproc.py   post-processing of C(r, t) (Sec. 2): spin projection to (J, M),
                A1+ projection over the cubic group, HAL QCD central potential.
  cpt.py        forward/backward (CPT) average of upper and lower components
                (Sec. 6).
"""
