"""FP64 CPU oracle of the photon path. Test infrastructure only."""
