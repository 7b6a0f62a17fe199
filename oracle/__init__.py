"""FP64 CPU oracle for the Hamiltonian ray tracing (HRT) hot path.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it. The product
path (the HIP library and its Python binding) never does, and it shares no code,
tables or constants with this package.

Everything here is plain, slow and written to be checked by eye against the
paper (Zhou et al., "A Hamiltonian, post-Born, three-dimensional, on-the-fly ray
tracing algorithm for gravitational lensing", arXiv:2405.12913):

* ``cosmo``        background expansion, comoving distance, linear growth (Sec. 2, Sec. 3.2)
* ``mesh``         cloud-in-cell paint / readout, FFT Poisson gradient (Sec. 2, Sec. 5.2)
* ``tables``       step schedule, lens shells and kick/drift factors (Sec. 3.1-3.2)
* ``integrator``   matter and ray kick-drift-kick steps (Eqs. symp_1-3, kick, drift; Alg. 1)
* ``observables``  distortion matrix and kappa/gamma/omega (Eqs. A, obs_first_set, obs_second_set)
* ``ic``           Gaussian initial conditions and 2LPT (Sec. 6.2; not part of the paper's method)
* ``pointmass``    point-lens deflection targets (Eqs. pointmass_analytic, pointmass_periodic)
* ``replicas``     per-replica transforms of the replicated light cone (Sec. 6.2)

Arrays are float64. Meshes are indexed ``[z, y, x]`` with the line of sight
along +z; particle and ray coordinates are ``(x, y, z)`` / ``(x, y)``.
"""
