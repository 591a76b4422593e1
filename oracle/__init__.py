"""CPU oracle for the trigger-station triplet selection.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import, call or link anything here; the
product library never does, and shares no code with it.
"""
