"""CPU oracle of the hide-and-seek step. Test infrastructure only."""
