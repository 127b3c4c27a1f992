"""Process generator: Feynman diagrams -> HIP device code and colour tables.

Built independently of any reference implementation: the diagram topology,
the colour reduction and the colour matrix are derived here and emitted as
straight-line FP64 device code (one event x one helicity per lane) plus an
exact integer colour matrix with a common denominator.
"""
