"""CPU oracle (test infrastructure only): plain FP64 reference of the
orthogonalization-free Rayleigh-Ritz path.  Imported only by tests/, the
smoke check and the CPU-baseline leg of bench.py."""
