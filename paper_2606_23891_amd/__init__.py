"""MI355X-native pack / interact / unpack for SPH (density, gradient, force).

Importing the package loads nothing native; the HIP library is opened on first
use through :mod:`paper_2606_23891_amd.sph` and fails loudly when it is missing.
"""
