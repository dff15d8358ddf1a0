"""CPU FP64 oracle for the method of polarized traces (Zepeda-Nunez & Demanet, 2014).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: it is used by the tests, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``.  It shares no code with the
GPU library (only the seeded input generators in ``synth`` feed both).

Modules
-------
assemble   -- PML profile, global 5-point operator, layer split, local operators
direct     -- sparse direct solve of the whole PML-padded system (the plain
              definition of the result the method reaches)
polarized  -- naive polarized-traces solve: local Green's trace blocks, the
              jump-condition system, Gauss-Seidel sweeps, flexible GMRES,
              reconstruction
plr        -- partitioned low-rank compression and its matrix-vector product

Everything is float64 / complex128.  Every function cites the passage of the
paper it follows.  Parity status of each function is recorded in its module
docstring ("pinned by ..." or "parity unpinned").
"""
