"""CPU oracle for GAME (Cavuoti et al., "Astrophysical data mining with GPU.
A case study: genetic classification of globular clusters").

This package is TEST INFRASTRUCTURE.  It is a plain, slow, obviously correct
restatement of what the paper's method computes, written from the paper's
equations:

* ``oracle.game``   - polynomial expansions (Eqs. 1, 8, 9), the pattern output
                      (Eq. 2), the error functions MSE / RMSE / TMSE
                      (Eqs. 3-5, 10), in float64.
* ``oracle.philox`` - the Philox4x64-10 counter-based generator (Salmon et al.,
                      SC'11), used for every random draw of the GA.
* ``oracle.ga``     - initialisation, ranking, elitism, tournament selection,
                      one-point crossover and Gaussian mutation (Sec. 2 option
                      list; Sec. 5 parameter list), and the training loop of
                      Sec. 4.1 (steps 1-4).
* ``oracle.mlp``    - the fitness-surrogate network, forward and backward, in
                      float64.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
imports it; the HIP path never imports this package.
"""
