"""CPU FP64 oracle for the ISM photochemistry + heating/cooling source step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path never does, and the oracle imports nothing from
the product package.

It follows Kim, Gong, Kim & Ostriker (arXiv:2210.08024):

* ``micro``    rate coefficients, heating, cooling, dust temperature and the
               equilibrium C/O/electron closure (Secs. 3-4).
* ``step``     the subcycled, operator-split source step (Sec. 6.1).
* ``columns``  six-ray diffuse-UV columns, shielding, N_eff and CR
               attenuation (Secs. 5.1-5.3).
* ``steady``   independent brute-force steady states (used as a pin).
* ``census``   the operation count of one substep (the step's roofline work).
* ``mlp``      FP64 reference forward/backward/Adam of the surrogate MLP.
* ``art``      adaptive ray tracing of point sources, its flux and the radiation
               force (Secs. 5.1, 6.2).
* ``sources``  the many-ray limit at cell centres (straight-line source maps).
* ``shield``   local shielding-length radiation and the shielded one-zone
               equilibrium (Sec. 7.1.2).
* ``slab``     the plane-parallel H I -> H2 transition (Sec. 7.3).

The tiny-dt checks integrate the same rate functions with scipy's DOP853 inside
the test itself.

Parity status of each function is stated in its docstring; where the paper
only cites a process (the tabulated and stand-in microphysics), the result is
"parity unpinned" beyond agreement with the HIP path.
"""
