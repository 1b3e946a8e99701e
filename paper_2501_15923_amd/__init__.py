"""MI355X-native heliospheric ideal-MHD hot path (Icarus 3.0, arXiv 2501.15923).

Import is light: the HIP library (libicarus_hip.so) is only loaded when a
Solver is created.  ``synth`` and ``configs`` produce the seeded inputs.
"""
__all__ = ["synth", "configs"]
