"""MI355X-native neural visibility queries (Neural Intersection Function).

Importing the package loads nothing; the HIP library is opened on first use
by :mod:`paper_2306_07191_amd.nif`."""
