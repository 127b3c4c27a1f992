"""Reference (oracle) implementation of the leading-order matrix element.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP path; the only thing both sides share is the seeded
phase-space generator, which holds no matrix-element arithmetic.

What it computes (the plain definition, written out slowly in float64):

    ME(p) = 1/IDEN * sum_{helicities} sum_{colours} |M(p, h, colours)|^2

for g g -> t tbar + k g, where M is the sum of all tree-level QCD Feynman
diagrams (tt~g, ggg, gggg vertices; Feynman-gauge gluon and top propagators).
The paper computes exactly this quantity as a quadratic form of colour-flow
("dual") amplitudes with a colour matrix, summed over helicities (the
pseudo-code of the monolithic kernel and the colour-sum equation J^H C J =
A^T C A + B^T C B); the paper prints no Feynman rules, so the vertices,
propagators and external states follow textbook QCD (Peskin & Schroeder,
ch. 16; helicity spinors in the chiral representation).

Modules
-------
kinematics   Minkowski algebra, gamma matrices, helicity spinors, polarisations
colour       colour strings and the exact colour matrix (Fierz reduction)
diagrams     enumeration of Feynman diagrams and their colour coefficients
me           diagram evaluation, dual amplitudes, colour and helicity sums
bg           colour-ordered Berends-Giele recursion (independent cross-check)
brute_colour explicit-colour sum with Gell-Mann matrices (cross-check)
closed_form  the analytic spin/colour-averaged g g -> t tbar result
"""
