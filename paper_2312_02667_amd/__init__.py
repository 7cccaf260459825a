"""MI355X-native parallel TEBD (pTEBD) layer with improved parallel MPS compression.

The package holds the ctypes binding to ``libptebd.so`` (``paper_2312_02667_amd.ptebd``),
the build step (``paper_2312_02667_amd.build``) and the seeded synthetic-input generators
(``paper_2312_02667_amd.inputs``).  Nothing is imported eagerly, so importing the package
never loads the native library.
"""

__all__ = ["inputs", "ptebd", "build"]
