"""CPU FP64 oracle for the AIM-accelerated GIBC surface-integral-equation method.

Test infrastructure only: this package may be imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``, and
by nothing else.  It shares no code with the HIP library (no kernels, headers,
tables or helpers); the two meet only through the seeded inputs in
``workloads/``.

Modules (each function cites the passage of Sharma & Triverio, "An Accelerated
Surface Integral Equation Method for the Electromagnetic Modeling of Dielectric
and Lossy Objects of Arbitrary Conductivity", IEEE TAP, arXiv:2003.11679 that it
follows):

* ``physics``   - complex permittivity, wavenumber, impedance (Sec. II, eq. kin/etain)
* ``rwg``       - RWG topology and basis functions (Sec. III-A)
* ``quad``      - collapsed Gauss-Legendre triangle rules
* ``static``    - closed-form 1/R potentials of a flat triangle
* ``mom``       - dense Galerkin L, K, X and excitation (Sec. III-A/B)
* ``solve``     - dense block and GIBC solves (eq. GIBCdef, GIBCsys)
* ``farfield``  - radiated far field and RCS (Sec. V-A)
* ``mie``       - Mie series for a homogeneous sphere (Sec. V-A reference)
* ``aim``       - AIM reference: grid, stencils, projection, convolution,
                  near list, precorrection (Sec. III-D-1, eq. AIM_Lin/AIM_Kin)
* ``bound``     - Lagrange interpolation error bound (Sec. IV, eq. Ddef)
* ``aefie``     - augmented EFIE and constraint preconditioner (Sec. III-E,
                  eq. sys)
"""
