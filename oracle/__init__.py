"""CPU oracle for the CC3 triples residual: test infrastructure only (see cc3_oracle.py)."""
