"""CPU FP64 oracle (test infrastructure only; see cheb_oracle.py)."""
