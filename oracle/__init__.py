"""CPU oracle of the 4pi track finding (test infrastructure only)."""
