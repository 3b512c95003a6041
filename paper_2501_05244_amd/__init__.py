"""MI355X-native NURSD / SRSD reconstruction (HIP kernels behind a C ABI).

    from paper_2501_05244_amd.api import Plan, plan_from_workload

The compute path is libnursd.so (built by paper_2501_05244_amd/build.py);
this package only marshals arguments to it.
"""
