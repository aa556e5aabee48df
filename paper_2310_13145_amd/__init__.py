"""MI355X-native UC-ACOPF two-level ADMM (HIP kernels behind a C-ABI).

Import ``paper_2310_13145_amd.ucac`` for the library binding and
``paper_2310_13145_amd.synth`` for seeded synthetic instances.
"""
