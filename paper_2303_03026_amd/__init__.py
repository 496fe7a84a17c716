"""MI355X-native GLM-MHD block-AMR hot path (arXiv 2303.03026, MPI-AMRVAC 3.0).

Importing the package loads nothing: ``paper_2303_03026_amd.amrvac`` is the
binding of the HIP library, ``paper_2303_03026_amd.inputs`` the seeded input
generator.
"""
