"""FP64 CPU oracle for ICNNM: test infrastructure only (tests, smoke check, benchmark CPU baseline)."""
