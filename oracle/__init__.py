"""Plain CPU oracle of the coupled lattice-Boltzmann / atom step (test infrastructure only)."""
