"""Explicit TE/TM wakefield time stepping (Dohlus & Zagorodnov) on MI355X.

The compute path is the C-ABI library ``libtete.so`` (HIP kernels for gfx950);
this package only marshals arguments to it.  See ``include/tete.h``.
"""
