# two-site honeycomb on an (i, j) index grid, t = 1, written for the tests:
# A(s) bonds to B(s), B(s - e_i), B(s - e_j); one field value per atom
dim 2
size 2
n_coeff_variable 1
nn -1 0
l0; 1|-1
l1;
nn 1 0
l0;
l1; 0|-1
nn 0 -1
l0; 1|-1
l1;
nn 0 1
l0;
l1; 0|-1
nn 0 0
l0; 0|v|0; 1|-1
l1; 0|-1;  1|v|0
