"""MI355X-native super-droplet coalescence (Sect. 5.1.4 of the libcloudph++ 0.2 paper).

Modules:
  sdm    -- ctypes binding of the C ABI (``include/sdm.h``) over ``libsdm.so``;
  synth  -- seeded synthetic super-droplet populations (inputs only, no method arithmetic);
  serve  -- continuous-batching request loop over the batch ABI;
  build  -- hipcc build of ``libsdm.so`` for gfx950.

Importing the package loads nothing; ``sdm.lib()`` loads the HIP library and raises
if it has not been built.
"""
