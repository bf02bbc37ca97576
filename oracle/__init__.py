"""FP64 CPU oracle of the ph-AFQMC walker step (test infrastructure only:
imported by tests, the smoke check and the benchmark's CPU baseline)."""
