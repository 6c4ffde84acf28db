"""MI355X-native dense H,S -> density-matrix path (ELSI 2.x, arXiv:1912.13403).

The compute path lives in the HIP library ``libhsdm.so`` built from ``csrc/``;
``paper_1912_13403_amd.hsdm`` is its thin Python binding.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["inputs"]
