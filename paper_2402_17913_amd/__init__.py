"""MI355X-native multigrid Poisson solver and projection step (Neural Physics, arXiv 2402.17913).

The compute path is the HIP library ``libneuphys.so`` (gfx950); this package
only marshals arguments to it.  Import the binding from
``paper_2402_17913_amd.binding``; ``paper_2402_17913_amd.inputs`` holds the
seeded synthetic workloads.
"""
