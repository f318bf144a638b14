"""CPU oracle of the fragment kMC hot path: test infrastructure only."""
