"""MI355X-native multiple-precision dense matrix multiplication (DD / QD).

The compute path is the HIP library ``libmpgemm.so`` built from ``csrc/``;
``paper_1710_01839_amd.mpgemm`` is its thin ctypes binding.  Importing this
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
