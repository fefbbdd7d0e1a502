"""MI355X (gfx950) blocked LU with tournament pivoting (COnfLUX hot path).

The compute path is the HIP library libcfx.so (C ABI in include/cfx.h);
``paper_2010_05975_amd.cfx`` marshals PyTorch tensors into it.  Importing the
package does not load the library; calling any entry point does, and fails
loudly if it has not been built.
"""
