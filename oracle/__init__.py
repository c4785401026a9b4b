"""FP64 CPU oracle of the PICsar step: test infrastructure only."""
