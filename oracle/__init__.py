"""FP64 CPU oracle of BERN-NN bound propagation (test infrastructure only)."""
