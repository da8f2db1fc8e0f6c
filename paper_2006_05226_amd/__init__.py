"""MI355X-native multilevel CC2 / CCSD (MLCC2, MLCCSD) on Cholesky vectors.

The compute path is the C-ABI library ``libmlcc.so`` (HIP kernels for gfx950);
``paper_2006_05226_amd.mlcc`` is its thin ctypes binding.  Importing the
package does not load the library.
"""
