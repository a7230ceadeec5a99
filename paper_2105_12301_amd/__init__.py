"""All-to-all convergent cross mapping (kEDM, Takahashi et al., PEARC '21) on MI355X.

The compute path is the HIP library ``libedm.so`` behind the C ABI of
``include/edm.h``; ``paper_2105_12301_amd.edm`` is its ctypes binding and
``paper_2105_12301_amd.synth`` holds the seeded input generators.
"""
