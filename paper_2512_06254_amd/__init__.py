"""MI355X (gfx950) TOI snapshot imager and FITrig stage behind the libtoi C ABI.

``paper_2512_06254_amd.toi`` holds the ctypes binding; ``build`` compiles the
HIP library in-tree.  Importing the package loads nothing.
"""
