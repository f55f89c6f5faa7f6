"""CPU oracle of the PIC-MCC column step -- test infrastructure only.

Imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark; never by the product package.
"""
