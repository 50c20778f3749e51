"""CPU oracle (test infrastructure only; see zc_oracle.py)."""
