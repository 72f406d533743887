"""Oracle: plain float64 CPU reference for the QSA-PIC hot path.

TEST INFRASTRUCTURE ONLY -- imported by tests/, by the package smoke check
and by the benchmark's CPU-baseline leg; never by the product path.
"""
