"""MI355X-native PRIEST: batched projection-guided sampling planner (HIP for gfx950).

Importing the package loads nothing native; the HIP library is loaded on the
first call into :mod:`paper_2309_08235_amd.priest`.
"""
