"""CPU oracle for the neural visibility path.  Test infrastructure only."""
