"""MI355X-native null-space-free eigensolver for 3-D Maxwell equations in chiral
and pseudochiral media (Chern, Hsieh, Huang, Lin, Wang).

* ``paper_1402_6297_amd.nsf``   -- ctypes binding of libnsf.so (include/nsf.h)
* ``paper_1402_6297_amd.media`` -- seeded synthetic media and k-paths
* ``paper_1402_6297_amd.build`` -- builds libnsf.so for gfx950 in-tree

Importing the package loads nothing; the HIP library is loaded on first use
and its absence raises.
"""
__all__ = ["nsf", "media", "build"]
