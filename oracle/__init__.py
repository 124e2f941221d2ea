"""FP64 CPU oracle for the WPCD three-body hot path (Pomerantsev, Kukulin, Rubtsova,
"Solving discretized Faddeev equations on a graphics processing unit").

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it. The product library
(``paper_1404_5253_amd``) never imports, calls or links anything here, and nothing here imports
the product: the two share no code, tables or constants. The only module both sides read is
``workloads.py`` (seeded synthetic inputs, none of the method's arithmetic).

Everything is plain NumPy/SciPy (plus SymPy's exact Wigner symbols and mpmath for pins) in
float64, written to be checked against the paper by eye rather than to be fast.

Module map (paper section / equation each follows):

* ``lattice``      free wave-packet bins, unit momentum weights (Sec. II.B.1, eq. pq; Appendix,
                   projection of plane waves onto WP states) and the nd kinematics.
* ``potential``    NN input: separable Yamaguchi and Malfliet-Tjon-type Yukawa sums in the free
                   WP basis (the v1 of eq. Ueq).
* ``pseudostates`` diagonalisation of h1 in the free WP basis (eq. exp_z) and the
                   scattering-WP bins.
* ``channels``     jj-coupled three-body channels (eq. qnum).
* ``recoupling``   spin-isospin-angular coefficients g (Appendix, eqs. ggaga and gal).
* ``mscheme``      independent m-scheme evaluation of the same angular function G (pin).
* ``perm``         P0 in the lattice basis: the Gauss rule on the polar (phi, x) form
                   (Appendix, final formula), plus a semi-analytic and a brute-force evaluation.
* ``resolvent``    the diagonal channel resolvent G1 in the SWP basis (eqs. dg1a, dg1b).
* ``solve``        the matrix Faddeev equation (eq. m_pvg) by iteration with Pade (Wynn epsilon)
                   summation, and by a direct sparse solve (pin).
* ``amplitude``    on-shell elastic amplitude (Sec. II.B.4), S-matrix, phase and inelasticity.
* ``pipeline``     end-to-end driver used by tests and the CPU baseline.

Readings of passages where the paper is silent or garbled are listed in the design doc; each is
also stated at the point of use below.
"""
