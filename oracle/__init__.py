"""Plain FP64 CPU oracle for DINO-accelerated geometric MCMC (Cao, O'Leary-Roseberry
& Ghattas, "Efficient geometric Markov chain Monte Carlo for nonlinear Bayesian
inversion enabled by derivative-informed neural operators", arXiv 2403.08220).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_2403_08220_amd``) never imports, links or executes anything here, and
nothing here imports the product path. The two share only the seeded input
generators in ``synth/``, which hold none of the method's arithmetic.

Modules, each written from the paper (sections/equations cited per function):

* ``philox``  - Philox4x64-10 counter-based generator (Salmon et al., SC'11) and the
  uniform / Box-Muller normal maps that both sides use for the draws of Alg. 1.
* ``prior``   - grid Matern prior (-gamma Lap + delta I)^-2, closed-form KLE basis
  (Sec. 4.2), encoder/decoder (eq. projector), complement variance.
* ``network`` - reduced-basis neural operator f_NN (eq. rb_dino): MLP and ResNet,
  exact GELU, reverse- and forward-mode reduced Jacobian.
* ``mcmc``    - surrogate misfit / reduced ppg / reduced ppGNH (Sec. 5.1), the
  surrogate mMALA proposal split (the splitting proposition of Sec. 5.3, eq. reduced_space_sampling), the
  reduced RN derivative and first-stage ratio (Sec. 5.4, eq. da_dino_trr_1),
  Alg. 1 first stage with the pCN complement move, N-step runs.
* ``stats``   - multichain ESS% (Sec. 6.2.2, eq. ess), Rao-Blackwellised posterior
  mean/variance, Wasserstein MPSRF (Sec. 6.2.1).

Precision: float64 throughout (the paper fixes no precision).

Pins (tests/test_oracle_*.py, marked "not gpu") tie every function to something
other than itself: numpy's Philox, dense eigh of the grid operator, central
finite differences, the textbook Gaussian MH ratio, closed-form Gaussian
posteriors for a linear surrogate, prior reversibility, quadrature on R^1/R^2
and AR(1) processes with known ESS.
"""
