"""MI355X-native collision step of the test-particle kinetic Monte Carlo
method (Sagert et al., arXiv:1210.8084).

The compute path is the HIP library built from ``csrc/`` and reached through
:mod:`paper_1210_8084_amd.tpkmc`; :mod:`paper_1210_8084_amd.workloads` draws
the seeded initial states.  Importing the package loads nothing native.
"""
