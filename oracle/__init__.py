"""FP64 CPU oracle of the WFB LBM-LES channel step -- test infrastructure only."""
