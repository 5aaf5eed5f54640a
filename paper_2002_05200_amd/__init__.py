"""MI355X-native batched X-drop seed extension (LOGAN, arXiv 2002.05200).

The package is deliberately import-light: ``synth`` (seeded synthetic read
pairs) imports only numpy, and the HIP binding lives in ``xdrop`` and is
loaded on first use.
"""

__all__ = ["synth", "xdrop"]
