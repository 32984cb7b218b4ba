"""MI355X-native localized-RI exact-exchange energy, forces and stress.

``paper_2412_11081_amd.lrx`` binds the HIP library (C-ABI in ``include/lrx.h``);
``paper_2412_11081_amd.synth`` builds seeded synthetic inputs.  Importing the
package loads nothing native; the binding loads ``liblrx.so`` on first use and
raises if it is missing.
"""
