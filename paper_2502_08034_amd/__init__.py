"""Steady state-of-charge solver for voxelised porous flow-battery electrodes on MI355X.

The HIP library (``csrc/``) is loaded lazily by ``paper_2502_08034_amd.socfv``; importing
this package does not touch the GPU.
"""
__all__ = ["inputs"]
