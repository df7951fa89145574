"""CPU FP64 checker for the monolithic GDSW / FGMRES path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or runs this
package; only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path: the only common
module is ``inputs`` (problem presets and seeded random numbers).

Every function follows a passage of the paper (Köhler & Rheinbach,
"Monolithic Multi-level Overlapping Schwarz Solvers for Fluid Problems"):

* ``stokes``         Section 2: weak Stokes form, Q2 velocity, eq. (2.1).
* ``decomposition``  Section 2.1: subdomains, overlap, interface Gamma and its
                     vertex/edge/face entities.
* ``gdsw``           eqs. (2.2)-(2.4): two-level monolithic GDSW preconditioner.
* ``threelevel``     eq. (2.5): three-level preconditioner.
* ``fgmres``         Tables 1-4 captions: FGMRES with a relative tolerance.
* ``conv``           dense FP64 3-D convolution network (learned local solve).
* ``counts``         closed-form and enumerated sizes behind Tables 1 and 2.

Pinned by ``tests/test_oracle_*.py``.  Parity status of each function is in
its module docstring.
"""
