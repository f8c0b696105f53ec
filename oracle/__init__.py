"""CPU FP64 oracle for the light-field renderer (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import this
package.  It shares no code with the HIP path (``paper_2407_14053_amd``) and never imports it.
"""
