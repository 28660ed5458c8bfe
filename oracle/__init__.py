"""FP64 CPU oracle for k-means|| -- test infrastructure only (tests/, the
smoke check and the benchmark's CPU-baseline leg).  The library never
imports it."""
