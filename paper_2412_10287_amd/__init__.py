"""Single-source two-way regular path queries on MI355X.

The engine is the C-ABI library ``librpq.so`` (HIP kernels for gfx950, declared
in ``include/rpq.h``); ``paper_2412_10287_amd.rpq`` is its ctypes binding and
``paper_2412_10287_amd.build`` compiles it. Importing the package does not load
the library; importing ``.rpq`` does, and fails if it is not built."""
